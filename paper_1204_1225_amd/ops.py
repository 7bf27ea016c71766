"""Python entry points over libkirchhoff.so (argument marshalling only).

Device memory and streams come from PyTorch; every step of migration,
demigration, counting and the float64 reductions runs in the HIP library.
A `DeviceProblem` holds the device-resident inputs of one problem (traces,
geometry, bins, grid and model tables) in the layouts of include/kirchhoff.h.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import (KmAntialias, KmGrid, KmLtable, KmProblem, KmTileInfo, KmTraces, KmTraveltime, KmTtable, KmWeight,
                   check)

_DTYPES = {"f32": _lib.KM_F32, "bf16": _lib.KM_BF16, "f16": _lib.KM_F16}
_PRECISIONS = {"fp32": _lib.KM_TIME_FP32, "extended": _lib.KM_TIME_EXTENDED}


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@dataclasses.dataclass
class DeviceProblem:
    """Device-resident inputs of one migration problem."""

    device: torch.device
    n_t: int
    dt: float
    t_first: float
    n_bins: int
    weight: int
    src: torch.Tensor       # float32 [n, 2]
    rec: torch.Tensor       # float32 [n, 2]
    bin: torch.Tensor       # int32 [n], nondecreasing
    x: torch.Tensor         # float32 [nx]
    y: torch.Tensor         # float32 [ny]
    t0sq: torch.Tensor      # float32 [nz]
    s2: torch.Tensor        # float32 [nz]
    r2: torch.Tensor        # float32 [nz]
    data: Optional[torch.Tensor] = None   # [n, n_t] float32, or int16 bit patterns of bf16 / f16
    scale: Optional[torch.Tensor] = None  # float32 [n] for 16-bit data
    dtype: str = "f32"
    ttab: Optional[torch.Tensor] = None   # float32 [n_h, nz] one-way times: table traveltimes (W = 1)
    tdh: float = 0.0
    # laterally varying tables: (gx0, gy0, gdx, gdy) of the node grid; ttab is then [n_gy, n_gx, n_h, nz]
    tgrid: Optional[tuple] = None
    tamp: Optional[torch.Tensor] = None   # float32, ttab's shape: one-way amplitudes (W = A_s A_r)
    aa: Optional[tuple] = None            # (dx, dy, max half-width): anti-alias triangle filter
    prec: str = "fp32"                    # time arithmetic: "fp32" or "extended" (km_time_precision)

    @property
    def n_traces(self) -> int:
        return int(self.src.shape[0])

    @property
    def nx(self) -> int:
        return int(self.x.shape[0])

    @property
    def ny(self) -> int:
        return int(self.y.shape[0])

    @property
    def nz(self) -> int:
        return int(self.t0sq.shape[0])

    @property
    def image_shape(self):
        return (self.n_bins, self.ny, self.nx, self.nz)

    def with_data(self, data: torch.Tensor, scale: Optional[torch.Tensor] = None, dtype: str = "f32"):
        return dataclasses.replace(self, data=data, scale=scale, dtype=dtype)

    # ctypes views -----------------------------------------------------------
    def c_traces(self, data: Optional[torch.Tensor] = None, dtype: Optional[str] = None,
                 scale: Optional[torch.Tensor] = None) -> KmTraces:
        d = self.data if data is None else data
        dt_name = self.dtype if dtype is None else dtype
        sc = (self.scale if data is None else scale) if dt_name != "f32" else None
        stride = int(d.stride(0)) if d is not None and d.dim() == 2 and d.numel() > 0 else self.n_t
        if d is not None:
            assert d.shape == (self.n_traces, self.n_t) and d.device == self.device
            assert d.numel() == 0 or d.stride(1) == 1
        return KmTraces(n_traces=self.n_traces, n_samples=self.n_t, dtype=_DTYPES[dt_name], trace_stride=stride,
                        t_first=self.t_first, dt=self.dt, data=_ptr(d), scale=_ptr(sc), src=_ptr(self.src),
                        rec=_ptr(self.rec), bin=_ptr(self.bin))

    def c_grid(self) -> KmGrid:
        return KmGrid(nx=self.nx, ny=self.ny, nz=self.nz, n_bins=self.n_bins, x=_ptr(self.x), y=_ptr(self.y))

    @property
    def c_prec(self) -> int:
        return _PRECISIONS[self.prec]

    def with_precision(self, prec: str):
        assert prec in _PRECISIONS
        return dataclasses.replace(self, prec=prec)

    def c_tt(self) -> KmTraveltime:
        return KmTraveltime(t0sq=_ptr(self.t0sq), s2=_ptr(self.s2), r2=_ptr(self.r2), time_precision=self.c_prec)

    def c_weight(self) -> KmWeight:
        return KmWeight(kind=int(self.weight))

    def c_aa(self) -> KmAntialias:
        assert self.aa is not None
        return KmAntialias(dx=float(self.aa[0]), dy=float(self.aa[1]), max_half=int(self.aa[2]))

    def c_table(self) -> KmTtable:
        assert self.ttab is not None and self.tgrid is None
        assert self.ttab.dim() == 2 and self.ttab.shape[1] == self.nz and self.ttab.is_contiguous()
        return KmTtable(n_h=int(self.ttab.shape[0]), dh=float(self.tdh), t=_ptr(self.ttab), r2=_ptr(self.r2),
                        time_precision=self.c_prec, amp=self._c_amp())

    def _c_amp(self):
        if self.tamp is None:
            return None
        assert self.tamp.shape == self.ttab.shape and self.tamp.is_contiguous()
        return _ptr(self.tamp)

    def c_ltable(self) -> KmLtable:
        assert self.ttab is not None and self.tgrid is not None
        assert self.ttab.dim() == 4 and self.ttab.shape[3] == self.nz and self.ttab.is_contiguous()
        n_gy, n_gx, n_h, _ = (int(v) for v in self.ttab.shape)
        gx0, gy0, gdx, gdy = (float(v) for v in self.tgrid)
        return KmLtable(n_h=n_h, dh=float(self.tdh), n_gx=n_gx, n_gy=n_gy, gx0=gx0, gy0=gy0, gdx=gdx, gdy=gdy,
                        t=_ptr(self.ttab), r2=_ptr(self.r2), time_precision=self.c_prec, amp=self._c_amp())


def to_device(problem, device="cuda", data=None, dtype: str = "f32", prec: str = "fp32") -> DeviceProblem:
    """Copy a survey problem's inputs to the GPU in the ABI layouts.

    Tables are converted to float32 (the ABI's table type).  dtype "bf16" /
    "f16" stores the traces with a per-trace scale (survey.quantise)."""
    from . import survey

    dev = torch.device(device)
    if dev.type == "cuda" and dev.index is None:
        dev = torch.device("cuda", torch.cuda.current_device())

    def f32(a):
        return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=dev)

    dp = DeviceProblem(device=dev, n_t=int(problem.n_t), dt=float(problem.dt), t_first=float(problem.t_first),
                       n_bins=int(problem.n_bins), weight=int(problem.weight), src=f32(problem.src),
                       rec=f32(problem.rec),
                       bin=torch.as_tensor(np.ascontiguousarray(problem.bin, dtype=np.int32), device=dev),
                       x=f32(problem.x), y=f32(problem.y), t0sq=f32(problem.t0sq), s2=f32(problem.s2),
                       r2=f32(problem.r2), prec=prec)
    if getattr(problem, "ttab", None) is not None:
        tgrid = getattr(problem, "tgrid", None)
        tamp = getattr(problem, "tamp", None)
        dp = dataclasses.replace(dp, ttab=f32(problem.ttab), tdh=float(problem.tdh),
                                 tgrid=None if tgrid is None else tuple(float(v) for v in tgrid),
                                 tamp=None if tamp is None else f32(tamp))
    if getattr(problem, "aa", None) is not None:
        dp = dataclasses.replace(dp, aa=tuple(problem.aa))
    d = problem.data if data is None else data
    if d is None:
        return dp
    if isinstance(d, torch.Tensor):
        if dtype != "f32":
            d = d.detach().cpu().numpy()
        else:
            return dp.with_data(d.to(device=dev, dtype=torch.float32).contiguous())
    if dtype == "f32":
        return dp.with_data(f32(d))
    bits, sig, _ = survey.quantise(np.asarray(d, dtype=np.float32), dtype)
    return dp.with_data(torch.as_tensor(bits.view(np.int16), device=dev), f32(sig), dtype)


def migrate(dp: DeviceProblem, data: Optional[torch.Tensor] = None, image: Optional[torch.Tensor] = None,
            accumulate: bool = False, tile: int = -1, dtype: Optional[str] = None,
            scale: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Eq. (1): image [n_bins, ny, nx, nz] float32 from the problem's traces
    (or `data`).  accumulate=True adds into `image`."""
    if image is None:
        image = torch.empty(dp.image_shape, dtype=torch.float32, device=dp.device)
        if accumulate:
            image.zero_()
    assert image.shape == dp.image_shape and image.dtype == torch.float32 and image.is_contiguous()
    tr = dp.c_traces(data, dtype if data is not None else None, scale)
    lib = _lib.load()
    if dp.tgrid is not None:
        check(lib.kirchhoff_migrate_ltable(ctypes.byref(tr), ctypes.byref(dp.c_grid()), ctypes.byref(dp.c_ltable()),
                                           _ptr(image), int(accumulate), int(tile),
                                           ctypes.c_void_p(_stream(dp.device))))
        return image
    if dp.ttab is not None:
        check(lib.kirchhoff_migrate_table(ctypes.byref(tr), ctypes.byref(dp.c_grid()), ctypes.byref(dp.c_table()),
                                          _ptr(image), int(accumulate), int(tile),
                                          ctypes.c_void_p(_stream(dp.device))))
        return image
    if dp.aa is not None:
        check(lib.kirchhoff_migrate_aa(ctypes.byref(tr), ctypes.byref(dp.c_grid()), ctypes.byref(dp.c_tt()),
                                       ctypes.byref(dp.c_weight()), ctypes.byref(dp.c_aa()), _ptr(image),
                                       int(accumulate), int(tile), ctypes.c_void_p(_stream(dp.device))))
        return image
    check(lib.kirchhoff_migrate(ctypes.byref(tr), ctypes.byref(dp.c_grid()), ctypes.byref(dp.c_tt()),
                                ctypes.byref(dp.c_weight()), _ptr(image), int(accumulate), int(tile),
                                ctypes.c_void_p(_stream(dp.device))))
    return image


def demigrate(dp: DeviceProblem, image: torch.Tensor, out: Optional[torch.Tensor] = None,
              accumulate: bool = False, tile: int = -1) -> torch.Tensor:
    """Transpose of migrate: float32 traces [n_traces, n_t] from an image."""
    assert image.shape == dp.image_shape and image.dtype == torch.float32 and image.is_contiguous()
    if out is None:
        out = torch.empty((dp.n_traces, dp.n_t), dtype=torch.float32, device=dp.device)
        if accumulate:
            out.zero_()
    tr = dp.c_traces(out, "f32")
    lib = _lib.load()
    if dp.tgrid is not None:
        check(lib.kirchhoff_demigrate_ltable(_ptr(image), ctypes.byref(dp.c_grid()), ctypes.byref(dp.c_ltable()),
                                             ctypes.byref(tr), int(accumulate), int(tile),
                                             ctypes.c_void_p(_stream(dp.device))))
        return out
    if dp.ttab is not None:
        check(lib.kirchhoff_demigrate_table(_ptr(image), ctypes.byref(dp.c_grid()), ctypes.byref(dp.c_table()),
                                            ctypes.byref(tr), int(accumulate), int(tile),
                                            ctypes.c_void_p(_stream(dp.device))))
        return out
    if dp.aa is not None:
        check(lib.kirchhoff_demigrate_aa(_ptr(image), ctypes.byref(dp.c_grid()), ctypes.byref(dp.c_tt()),
                                         ctypes.byref(dp.c_weight()), ctypes.byref(dp.c_aa()), ctypes.byref(tr),
                                         int(accumulate), int(tile), ctypes.c_void_p(_stream(dp.device))))
        return out
    check(lib.kirchhoff_demigrate(_ptr(image), ctypes.byref(dp.c_grid()), ctypes.byref(dp.c_tt()),
                                  ctypes.byref(dp.c_weight()), ctypes.byref(tr), int(accumulate), int(tile),
                                  ctypes.c_void_p(_stream(dp.device))))
    return out


def _plain_only(dp: DeviceProblem, what: str) -> None:
    """Raise for problems whose operator the call does not implement."""
    if dp.ttab is not None or dp.aa is not None:
        raise _lib.KirchhoffError(_lib.KM_E_UNSUPPORTED,
                                  f"{what}: table traveltimes and the anti-alias filter are not supported here")


def count(dp: DeviceProblem, aperture_only: bool = False):
    """(n_aperture, n_effective) of Eq. (2) from the counting kernel.  The
    aperture test does not depend on the traveltime kind, so with
    aperture_only=True any problem is accepted and (n_aperture, None) is
    returned; n_effective needs the square-root times of a plain problem."""
    if not aperture_only:
        _plain_only(dp, "count")
    c = torch.empty(2, dtype=torch.int64, device=dp.device)
    tr = dp.c_traces()
    lib = _lib.load()
    check(lib.km_count_contributions(ctypes.byref(tr), ctypes.byref(dp.c_grid()), ctypes.byref(dp.c_tt()),
                                     _ptr(c), ctypes.c_void_p(_stream(dp.device))))
    v = c.cpu().tolist()
    return int(v[0]), (None if aperture_only else int(v[1]))


def count_host(problem, n_threads: int = 0):
    """Exact (n_aperture, n_effective) of Eq. (2), counted on the host by the
    library from host (numpy) copies of a problem's geometry and float32
    tables: problem has src, rec, bin, x, y, t0sq, s2, r2, n_t, dt, t_first,
    n_bins (a survey problem or anything with those attributes)."""
    keep = {k: np.ascontiguousarray(getattr(problem, k), dtype=np.float32)
            for k in ("src", "rec", "x", "y", "t0sq", "s2", "r2")}
    keep["bin"] = np.ascontiguousarray(problem.bin, dtype=np.int32)
    n = int(keep["src"].shape[0])
    nz = int(keep["t0sq"].shape[0])
    assert keep["rec"].shape == (n, 2) and keep["bin"].shape == (n,)
    assert keep["s2"].shape == (nz,) and keep["r2"].shape == (nz,)

    def ptr(a):
        return ctypes.c_void_p(a.ctypes.data)

    tr = KmTraces(n_traces=n, n_samples=int(problem.n_t), dtype=_lib.KM_F32, trace_stride=int(problem.n_t),
                  t_first=float(problem.t_first), dt=float(problem.dt), data=None, scale=None, src=ptr(keep["src"]),
                  rec=ptr(keep["rec"]), bin=ptr(keep["bin"]))
    g = KmGrid(nx=int(keep["x"].shape[0]), ny=int(keep["y"].shape[0]), nz=nz, n_bins=int(problem.n_bins),
               x=ptr(keep["x"]), y=ptr(keep["y"]))
    tt = KmTraveltime(t0sq=ptr(keep["t0sq"]), s2=ptr(keep["s2"]), r2=ptr(keep["r2"]), time_precision=0)
    na, ne = ctypes.c_int64(0), ctypes.c_int64(0)
    check(_lib.load().km_count_contributions_host(ctypes.byref(tr), ctypes.byref(g), ctypes.byref(tt),
                                                  int(n_threads), ctypes.byref(na), ctypes.byref(ne)))
    return int(na.value), int(ne.value)


def dot_f64(a: torch.Tensor, b: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """float64 device scalar sum(a * b) of two float32 tensors of equal size."""
    assert a.dtype == torch.float32 and b.dtype == torch.float32 and a.numel() == b.numel()
    assert a.is_contiguous() and b.is_contiguous()
    if out is None:
        out = torch.empty((), dtype=torch.float64, device=a.device)
    check(_lib.load().km_dot_f64(_ptr(a), _ptr(b), a.numel(), _ptr(out), ctypes.c_void_p(_stream(a.device))))
    return out


def axpby(alpha: float, x: torch.Tensor, beta: float, y: torch.Tensor) -> torch.Tensor:
    """y = alpha x + beta y in place (float32)."""
    assert x.dtype == torch.float32 and y.dtype == torch.float32 and x.numel() == y.numel()
    assert x.is_contiguous() and y.is_contiguous()
    check(_lib.load().km_axpby(float(alpha), _ptr(x), float(beta), _ptr(y), y.numel(),
                               ctypes.c_void_p(_stream(y.device))))
    return y


def trace_filter(traces: torch.Tensor, taps: torch.Tensor, center: int, adjoint: bool = False,
                 out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """FIR pre-filter of every row of traces [n, n_samples] (float32, row
    stride taken from the tensor): forward out[n] = sum_k h[k] in[n + c - k],
    adjoint the transpose.  out may be traces itself."""
    assert traces.dtype == torch.float32 and traces.dim() == 2 and traces.stride(1) == 1
    assert taps.dtype == torch.float32 and taps.dim() == 1 and taps.is_contiguous() and taps.device == traces.device
    if out is None:
        out = torch.empty_like(traces, memory_format=torch.contiguous_format)
    assert out.shape == traces.shape and out.stride(1) == 1
    n, ns = traces.shape
    check(_lib.load().km_trace_filter(_ptr(traces), traces.stride(0) if n else ns, _ptr(out),
                                      out.stride(0) if n else ns, n, ns, _ptr(taps), taps.numel(), int(center),
                                      1 if adjoint else 0, ctypes.c_void_p(_stream(traces.device))))
    return out


def stack_offsets(image: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Sum of the offset images image[n_bins, ...] over the bins (float32)."""
    assert image.dtype == torch.float32 and image.is_contiguous() and image.dim() >= 1
    if out is None:
        out = torch.empty(image.shape[1:], dtype=torch.float32, device=image.device)
    assert out.is_contiguous() and out.numel() * image.shape[0] == image.numel()
    check(_lib.load().km_stack_offsets(_ptr(image), image.shape[0], out.numel(), _ptr(out),
                                       ctypes.c_void_p(_stream(image.device))))
    return out


def cig_moveout(image: torch.Tensor, offsets: Optional[torch.Tensor] = None, max_lag: int = 12, z_lo: int = 0,
                z_hi: Optional[int] = None, want_stack: bool = True, want_peak: bool = True):
    """Moveout of the common-image gathers of image[n_bins, ny, nx, nz] against
    their stack: returns (stack, shift, peak, curvature); stack / peak are
    None when not wanted, curvature is None without offsets (float32 [n_bins]
    bin-centre offsets on the image's device)."""
    assert image.dtype == torch.float32 and image.is_contiguous() and image.dim() == 4
    nb, ny, nx, nz = image.shape
    dev = image.device
    z_hi = nz if z_hi is None else z_hi
    stack = torch.empty((ny, nx, nz), dtype=torch.float32, device=dev) if want_stack else None
    shift = torch.empty((nb, ny, nx), dtype=torch.float32, device=dev)
    peak = torch.empty((nb, ny, nx), dtype=torch.float32, device=dev) if want_peak else None
    curv = None
    if offsets is not None:
        assert offsets.dtype == torch.float32 and offsets.numel() == nb and offsets.device == dev
        offsets = offsets.contiguous()
        curv = torch.empty((ny, nx), dtype=torch.float32, device=dev)
    g = KmGrid(nx=nx, ny=ny, nz=nz, n_bins=nb, x=None, y=None)
    check(_lib.load().km_cig_moveout(_ptr(image), ctypes.byref(g), _ptr(offsets), max_lag, z_lo, z_hi, _ptr(stack),
                                     _ptr(shift), _ptr(peak), _ptr(curv), ctypes.c_void_p(_stream(dev))))
    return stack, shift, peak, curv


def tile_count(op: int) -> int:
    return int(_lib.load().km_tile_count(op))


def tile_describe(op: int, tile: int) -> dict:
    info = KmTileInfo()
    check(_lib.load().km_tile_describe(op, tile, ctypes.byref(info)))
    return {f: int(getattr(info, f)) for f, _ in KmTileInfo._fields_}


def tile_levels(op: int) -> int:
    return int(_lib.load().km_tile_levels(op))


def tiles(op: int, dp: Optional["DeviceProblem"] = None):
    """Every valid tile of op: compiled shape + 64 * level.  Given a problem,
    only the tiles that apply to it: the 16-bit staging levels of migrate take
    16-bit traces with float32 time and no anti-alias filter."""
    out = []
    s16_ok = dp is None or (dp.dtype != "f32" and dp.prec == "fp32" and dp.aa is None)
    for lv in range(tile_levels(op)):
        for sh in range(tile_count(op)):
            t = sh + 64 * lv
            info = KmTileInfo()
            if _lib.load().km_tile_describe(op, t, ctypes.byref(info)) == _lib.KM_OK and (s16_ok or not info.lds16):
                out.append(t)
    return out


KIND_DSR, KIND_TABLE, KIND_AA, KIND_LTABLE = 0, 1, 2, 3


def problem_kind(dp: DeviceProblem) -> int:
    if dp.tgrid is not None:
        return KIND_LTABLE
    return KIND_TABLE if dp.ttab is not None else KIND_AA if dp.aa is not None else KIND_DSR


def tune(op: int, dp: DeviceProblem, image: torch.Tensor, traces_out: Optional[torch.Tensor] = None,
         reps: int = 2):
    """Time every tile of op (0 migrate, 1 demigrate) on dp (any traveltime
    kind) and record the fastest for its class; returns (tile, ms).  For op 0
    `image` is overwritten with the migration; for op 1 `image` is the input
    and `traces_out` (float32 [n_traces, n_t]) is overwritten."""
    best, ms = ctypes.c_int32(-1), ctypes.c_float(0.0)
    tr = dp.c_traces() if op == 0 else dp.c_traces(traces_out, "f32")
    if dp.tgrid is not None:
        check(_lib.load().km_tune_ltable(op, ctypes.byref(tr), ctypes.byref(dp.c_grid()), ctypes.byref(dp.c_ltable()),
                                         _ptr(image), int(reps), ctypes.c_void_p(_stream(dp.device)),
                                         ctypes.byref(best), ctypes.byref(ms)))
        return int(best.value), float(ms.value)
    tab = ctypes.byref(dp.c_table()) if dp.ttab is not None else None
    aa = ctypes.byref(dp.c_aa()) if dp.aa is not None else None
    check(_lib.load().km_tune(op, ctypes.byref(tr), ctypes.byref(dp.c_grid()), ctypes.byref(dp.c_tt()),
                              ctypes.byref(dp.c_weight()), tab, aa, _ptr(image), int(reps),
                              ctypes.c_void_p(_stream(dp.device)), ctypes.byref(best), ctypes.byref(ms)))
    return int(best.value), float(ms.value)


def tune_lookup(op: int, dp: DeviceProblem) -> int:
    """The tile recorded for dp's class (-1 if none)."""
    return int(_lib.load().km_tune_lookup(op, _DTYPES[dp.dtype], problem_kind(dp), dp.c_prec, dp.nz, dp.n_t))


def probe_issue(kind: int, n_waves: int = 8192, iters: int = 4096) -> float:
    """ms of the issue-rate probe (kind 0 fma, 1 sqrt, 2 rcp)."""
    ms = ctypes.c_float(0.0)
    check(_lib.load().km_probe_issue(kind, n_waves, iters, ctypes.c_void_p(_stream(torch.device("cuda"))),
                                     ctypes.byref(ms)))
    return float(ms.value)


def _c_problems(problems, images):
    assert len(problems) == len(images) and len(problems) > 0
    arr = (KmProblem * len(problems))()
    for k, (dp, img) in enumerate(zip(problems, images)):
        _plain_only(dp, "batched migration")
        assert img.shape == dp.image_shape and img.dtype == torch.float32 and img.is_contiguous()
        arr[k] = KmProblem(traces=dp.c_traces(), grid=dp.c_grid(), tt=dp.c_tt(), weight=dp.c_weight(),
                           image=_ptr(img))
    return arr


def batch_migrate_static(problems, images, tile: int = -1) -> None:
    """One batched migration of many problems that allocates no device memory
    (km_batch_migrate_static: the work list lives in the library's static
    scratch array).  Overwrites every image; calls on one GPU must not overlap."""
    arr = _c_problems(problems, images)
    dev = problems[0].device
    check(_lib.load().km_batch_migrate_static(arr, len(problems), int(tile), ctypes.c_void_p(_stream(dev))))


class Batch:
    """Many problems migrated by one persistent, graph-captured launch."""

    def __init__(self, problems, images, tile: int = -1):
        self._keep = (list(problems), list(images))
        self._arr = arr = _c_problems(problems, images)
        self._h = ctypes.c_void_p()
        dev = problems[0].device
        check(_lib.load().km_batch_create(arr, len(problems), 0, int(tile), ctypes.c_void_p(_stream(dev)),
                                          ctypes.byref(self._h)))
        self.device = dev

    def run(self):
        check(_lib.load().km_batch_run(self._h, ctypes.c_void_p(_stream(self.device))))

    def info(self):
        n, w = ctypes.c_int64(0), ctypes.c_int32(0)
        check(_lib.load().km_batch_info(self._h, ctypes.byref(n), ctypes.byref(w)))
        return int(n.value), int(w.value)

    def close(self):
        if self._h:
            check(_lib.load().km_batch_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
