"""Seeded synthetic seismic surveys: the inputs of the Kirchhoff migration operator.

The operator of Eq. (1) (Section 3 of "Distributed computing of Seismic Imaging
Algorithms") maps recorded traces D(x_s, x_r, t) to offset-binned images
I(x, X).  Everything it is *given* is built here, and nothing more:

* acquisition geometry: source and receiver positions of every trace
  (Section 2: shots, geophones, traces, shot records);
* the offset-bin label of each trace, i.e. the discretised delta(X - |x_s - x_r|)
  of Eq. (1), with traces sorted by bin;
* the traveltime model as per-depth tables: T(x, x_s) = sqrt(t0(z)^2 + s2(z) h^2)
  with h the horizontal source (or receiver) distance, the double-square-root
  form used for prestack time migration.  Eq. (1) takes the propagation times
  "in the model" as given; these tables are that model;
* the aperture table r2(z) (largest squared horizontal distance still "close
  enough", Eq. (2)), rounded once to float32 so that every consumer takes the
  same in/out decision;
* trace samples made by forward modelling of point scatterers with a Ricker
  wavelet, optionally with Gaussian noise, or plain N(0, 1) samples;
* storage conversion of traces to bfloat16 / float16 with a per-trace scale.

This module contains no migration arithmetic (no time-to-sample interpolation,
no weighting of data, no summation into an image).  It is shared by the FP64
reference checker of the tests and by the GPU library's callers, and imports
neither.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

WEIGHT_UNIT = 0
WEIGHT_COSCOS = 1


@dataclasses.dataclass
class Problem:
    """One migration problem.  Arrays are numpy unless noted.

    Layout conventions (shared with the C ABI):
      src, rec : float32 [n_traces, 2]  (x, y) in metres
      bin      : int32   [n_traces], nondecreasing (traces grouped by bin)
      data     : float32 [n_traces, n_t] (sample-fastest) or None
      x, y     : float32 image coordinates; y has one entry for a 2D line
      z        : float64 image depths (z[iz] = (iz + 1) * dz)
      t0sq, s2 : float64 [nz] traveltime tables (s^2, s^2/m^2)
      r2       : float32 [nz] aperture table (m^2)
      image    : [n_bins][ny][nx][nz]
    """

    name: str
    src: np.ndarray
    rec: np.ndarray
    bin: np.ndarray
    data: Optional[np.ndarray]
    n_t: int
    dt: float
    t_first: float
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    n_bins: int
    t0sq: np.ndarray
    s2: np.ndarray
    r2: np.ndarray
    weight: int = WEIGHT_COSCOS
    velocity: tuple = ("const", 2000.0)
    aperture_deg: float = 45.0
    offset_bin_width: float = 0.0
    scatterers: Optional[np.ndarray] = None  # [m, 3] x, y, z of modelled point scatterers
    diffractor_nodes: Optional[np.ndarray] = None  # [m, 3] (ix, iy, iz) grid nodes
    meta: dict = dataclasses.field(default_factory=dict)
    # optional one-way traveltime table [n_h][nz] (seconds at h = ih * tdh), replacing t0sq / s2
    ttab: Optional[np.ndarray] = None
    tdh: float = 0.0
    # laterally varying tables: (gx0, gy0, gdx, gdy) of the node grid X_i = gx0 + i gdx,
    # Y_j = gy0 + j gdy; ttab is then [n_gy][n_gx][n_h][nz], one table per node
    tgrid: Optional[tuple] = None
    # optional one-way amplitudes of the table traveltimes (same layout as ttab): W = A_s A_r instead of 1
    tamp: Optional[np.ndarray] = None
    # optional anti-alias triangle filter: (dx, dy, largest half-width in samples)
    aa: Optional[tuple] = None

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
        return int(self.z.shape[0])

    @property
    def image_shape(self):
        return (self.n_bins, self.ny, self.nx, self.nz)

    def bin_ranges(self) -> np.ndarray:
        """CSR offsets: traces of bin b are [off[b], off[b+1])."""
        return np.searchsorted(self.bin, np.arange(self.n_bins + 1), side="left").astype(np.int64)

    def subset(self, idx) -> "Problem":
        """Problem restricted to the traces idx (kept in bin order)."""
        idx = np.sort(np.asarray(idx, dtype=np.int64))
        return dataclasses.replace(
            self,
            src=self.src[idx].copy(),
            rec=self.rec[idx].copy(),
            bin=self.bin[idx].copy(),
            data=None if self.data is None else self.data[idx].copy(),
        )


# ---------------------------------------------------------------------------
# Traveltime model tables (inputs of the operator)
# ---------------------------------------------------------------------------

def traveltime_tables(z: np.ndarray, velocity: tuple):
    """Per-depth tables (t0^2, s2) of T = sqrt(t0^2 + s2 * h^2), FP64.

    velocity = ("const", v):          t0 = z / v, s2 = 1 / v^2 (exact straight ray).
    velocity = ("linear", v0, k):     v(z) = v0 + k z with straight-ray RMS
        traveltimes: t0 is the one-way vertical time integral of dz / v,
        t0 = ln(1 + k z / v0) / k, and s2 = 1 / v_rms^2 with
        v_rms^2 = (1/t0) * integral_0^t0 v(t)^2 dt = (v(z)^2 - v0^2) / (2 k t0).
    """
    z = np.asarray(z, dtype=np.float64)
    kind = velocity[0]
    if kind == "const":
        v = float(velocity[1])
        t0 = z / v
        s2 = np.full_like(z, 1.0 / (v * v))
    elif kind == "linear":
        v0, k = float(velocity[1]), float(velocity[2])
        t0 = np.log1p(k * z / v0) / k
        vz = v0 + k * z
        with np.errstate(invalid="ignore", divide="ignore"):
            vrms2 = (vz * vz - v0 * v0) / (2.0 * k * t0)
        vrms2 = np.where(t0 > 0, vrms2, v0 * v0)
        s2 = 1.0 / vrms2
    else:
        raise ValueError(f"unknown velocity model {velocity!r}")
    return t0 * t0, s2


def curved_ray_time(h, z, v0: float, k: float):
    """One-way time of the curved (circular-arc) ray from a surface point to a
    point at horizontal distance h and depth z in v(z) = v0 + k z, FP64:
    T = acosh(1 + k^2 (h^2 + z^2) / (2 v0 v(z))) / k  (straight ray r / v0 at k = 0),
    with acosh(1 + e) evaluated as log1p(e + sqrt(e (e + 2)))."""
    h = np.asarray(h, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    if k == 0.0:
        return np.sqrt(h * h + z * z) / v0
    e = k * k * (h * h + z * z) / (2.0 * v0 * (v0 + k * z))
    return np.log1p(e + np.sqrt(e * (e + 2.0))) / k  # acosh(1 + e) without cancellation at small e


def curved_ray_table(z, v0: float, k: float, dh: float, n_h: int) -> np.ndarray:
    """ttab[ih][iz] = curved_ray_time(ih dh, z[iz]) rounded once to float32."""
    h = dh * np.arange(n_h, dtype=np.float64)
    return curved_ray_time(h[:, None], np.asarray(z, np.float64)[None, :], v0, k).astype(np.float32)


def curved_ray_amplitude_table(z, v0: float, k: float, dh: float, n_h: int) -> np.ndarray:
    """amp[ih][iz] = t0 / T^2 with T = curved_ray_time(ih dh, z[iz]) and t0 =
    T(0, z[iz]) (cos / T of the leg, cos = t0 / T), rounded once to float32.
    For constant velocity the product over the two legs is the square-root
    form's cos cos / (T_s T_r) weight exactly."""
    h = dh * np.arange(n_h, dtype=np.float64)
    zz = np.asarray(z, np.float64)[None, :]
    T = curved_ray_time(h[:, None], zz, v0, k)
    t0 = curved_ray_time(0.0, zz, v0, k)
    return (t0 / (T * T)).astype(np.float32)


def with_curved_ray_table(problem: "Problem", dh: float = 10.0, n_h: Optional[int] = None,
                          amplitude: bool = False) -> "Problem":
    """The problem with its traveltimes replaced by the curved-ray table of its
    linear (or constant) velocity model, covering every in-aperture leg;
    weight becomes W = 1, or with amplitude=True the product of the legs'
    curved_ray_amplitude_table values."""
    vel = problem.velocity
    v0, k = (float(vel[1]), 0.0) if vel[0] == "const" else (float(vel[1]), float(vel[2]))
    if n_h is None:
        hmax = float(np.sqrt(np.max(problem.r2.astype(np.float64))))
        n_h = int(np.ceil(hmax / dh)) + 2
    tab = curved_ray_table(problem.z, v0, k, dh, n_h)
    amp = curved_ray_amplitude_table(problem.z, v0, k, dh, n_h) if amplitude else None
    return dataclasses.replace(problem, ttab=tab, tdh=float(dh), tamp=amp, weight=WEIGHT_UNIT)


def lateral_v0(v0: float, gx: float, gy: float, xc: float, yc: float):
    """Surface velocity of a laterally varying medium v(x, y, z) = v0(x, y) + k z
    with v0(x, y) = v0 + gx (x - xc) + gy (y - yc) (a plane; FP64)."""
    return lambda x, y: v0 + gx * (np.asarray(x, np.float64) - xc) + gy * (np.asarray(y, np.float64) - yc)


def with_lateral_tables(problem: "Problem", v0_at, k: float, gx0: float, gy0: float, gdx: float, gdy: float,
                        n_gx: int, n_gy: int, dh: float = 10.0, n_h: Optional[int] = None,
                        amplitude: bool = False) -> "Problem":
    """The problem with laterally varying table traveltimes: below node
    (X_i, Y_j) = (gx0 + i gdx, gy0 + j gdy) the medium is taken as the depth-only
    v(z) = v0_at(X_i, Y_j) + k z, and the node's table holds its curved-ray
    times, ttab[j][i][ih][iz] = curved_ray_time(ih dh, z[iz]; v0_at(X_i, Y_j), k)
    rounded once to float32 (the local one-dimensional medium under each node).
    n_h covers every in-aperture leg by default; weight becomes W = 1, or with
    amplitude=True the product of the legs' amplitudes, each node holding its
    medium's curved_ray_amplitude_table."""
    if n_h is None:
        hmax = float(np.sqrt(np.max(problem.r2.astype(np.float64))))
        n_h = int(np.ceil(hmax / dh)) + 2
    X = gx0 + gdx * np.arange(n_gx, dtype=np.float64)
    Y = gy0 + gdy * np.arange(n_gy, dtype=np.float64)
    tab = np.empty((n_gy, n_gx, n_h, problem.nz), dtype=np.float32)
    amp = np.empty_like(tab) if amplitude else None
    for j in range(n_gy):
        for i in range(n_gx):
            v0 = float(v0_at(X[i], Y[j]))
            tab[j, i] = curved_ray_table(problem.z, v0, k, dh, n_h)
            if amplitude:
                amp[j, i] = curved_ray_amplitude_table(problem.z, v0, k, dh, n_h)
    return dataclasses.replace(problem, ttab=tab, tdh=float(dh), tamp=amp,
                               tgrid=(float(gx0), float(gy0), float(gdx), float(gdy)), weight=WEIGHT_UNIT)


SURVEY3D_LATERAL_V0 = (1500.0, 0.05, -0.04, 2500.0, 2500.0)  # v0, d v0 / dx, d v0 / dy, centre x, y


def with_survey3d_lateral_tables(p: "Problem", dh: float = 10.0) -> "Problem":
    """The 3D survey's laterally varying model: v(x, y, z) = v0(x, y) + 0.5 z
    with v0 = 1500 + 0.05 (x - 2500) - 0.04 (y - 2500) m/s (about 1420 to 1580
    over the image), tables of curved rays under each node of a 9 x 9 grid at
    400 m (900 .. 4100 m in x and y, covering the image), rows every dh m."""
    v0_at = lateral_v0(*SURVEY3D_LATERAL_V0)
    return with_lateral_tables(p, v0_at, 0.5, 900.0, 900.0, 400.0, 400.0, 9, 9, dh=dh)


def aperture_table(t0sq: np.ndarray, s2: np.ndarray, aperture_deg: float) -> np.ndarray:
    """r2[iz] = tan^2(theta_max) * t0^2 / s2, rounded once to float32.

    A leg of horizontal length h is inside the aperture at depth iz iff
    h^2 <= r2[iz]; for straight rays this is 'ray angle from vertical
    <= theta_max'.  theta >= 90 degrees means no aperture limit.
    """
    if aperture_deg >= 90.0:
        return np.full(t0sq.shape, np.finfo(np.float32).max, dtype=np.float32)
    tan2 = math.tan(math.radians(aperture_deg)) ** 2
    return (tan2 * t0sq / s2).astype(np.float32)


def offset_bins(src: np.ndarray, rec: np.ndarray, width: float, n_bins: int) -> np.ndarray:
    """bin = min(floor(|x_s - x_r| / width), n_bins - 1), |.| in FP64."""
    h = np.hypot(src[:, 0].astype(np.float64) - rec[:, 0], src[:, 1].astype(np.float64) - rec[:, 1])
    return np.minimum(np.floor(h / width), n_bins - 1).astype(np.int32)


def _sort_by_bin(src, rec, bins, extra=None):
    order = np.argsort(bins, kind="stable")
    out = [src[order], rec[order], bins[order]]
    if extra is not None:
        out.append(extra[order])
    return out


# ---------------------------------------------------------------------------
# Trace synthesis
# ---------------------------------------------------------------------------

def ricker(t, f_peak: float):
    """Zero-phase Ricker wavelet (1 - 2 pi^2 f^2 t^2) exp(-pi^2 f^2 t^2)."""
    a = (math.pi * f_peak * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def _leg_time_and_cos(velocity, sx, sy, rz, px, py):
    """Straight-ray one-way time and cos(angle from vertical) for legs from
    surface points (sx, sy) to scatterers (px, py, rz).  Arrays broadcast; FP64.

    Constant velocity uses the Euclidean path length (independent of the
    table form); v(z) uses the RMS double-square-root model of the tables."""
    import torch

    h2 = (px - sx) ** 2 + (py - sy) ** 2
    if velocity[0] == "const":
        v = float(velocity[1])
        dist = torch.sqrt(h2 + rz * rz)
        return dist / v, rz / dist
    v0, k = float(velocity[1]), float(velocity[2])
    t0 = torch.log1p(k * rz / v0) / k
    vz = v0 + k * rz
    vrms2 = (vz * vz - v0 * v0) / (2.0 * k * t0)
    T = torch.sqrt(t0 * t0 + h2 / vrms2)
    return T, t0 / T


def model_scatterers(problem: Problem, scat: np.ndarray, f_peak: float = 25.0,
                     device=None, chunk: int = 4096, half_width_s: float = 0.08, rays: str = "straight",
                     v0_at=None):
    """Trace samples from point scatterers: D_j(t) = sum_k a_kj r(t - tau_kj).

    tau_kj = source-leg + receiver-leg time, a_kj the obliquity/spreading
    factor cos_s cos_r / (T_s T_r) normalised per scatterer to a maximum of 1
    over all traces.  rays = "straight": straight rays (Euclidean for constant
    v, the RMS model for v(z)); rays = "curved": the exact circular-arc ray
    times of v(z) = v0 + k z with a_kj = 1 / (T_s T_r) normalised the same way.
    With v0_at (a function of (x, y)), curved rays see below each scatterer the
    depth-only medium v0_at(x_k, y_k) + k z (a laterally varying medium taken
    one-dimensional under the image point, as the lateral tables take it).
    Returns float32 [n, n_t] as a torch tensor on `device` (default CPU).
    """
    import torch

    dev = torch.device(device) if device is not None else torch.device("cpu")
    n, nt = problem.n_traces, problem.n_t
    dt, tf = problem.dt, problem.t_first
    src = torch.as_tensor(problem.src, dtype=torch.float64, device=dev)
    rec = torch.as_tensor(problem.rec, dtype=torch.float64, device=dev)
    sc = torch.as_tensor(np.asarray(scat, dtype=np.float64), device=dev)
    m = sc.shape[0]
    out = torch.zeros(n * nt, dtype=torch.float32, device=dev)
    if m == 0 or n == 0:
        return out.view(n, nt)
    px, py, pz = sc[:, 0][None, :], sc[:, 1][None, :], sc[:, 2][None, :]

    vel = problem.velocity
    v0, kg = (float(vel[1]), 0.0) if vel[0] == "const" else (float(vel[1]), float(vel[2]))
    if v0_at is not None:
        sc_np = np.asarray(scat, dtype=np.float64)
        v0 = torch.as_tensor(np.asarray(v0_at(sc_np[:, 0], sc_np[:, 1]), np.float64), device=dev)[None, :]

    def curved(sx, sy):
        h2 = (px - sx) ** 2 + (py - sy) ** 2
        if kg == 0.0:
            return torch.sqrt(h2 + pz * pz) / v0
        e = kg * kg * (h2 + pz * pz) / (2.0 * v0 * (v0 + kg * pz))
        return torch.log1p(e + torch.sqrt(e * (e + 2.0))) / kg

    def legs(j0, j1):
        if rays == "curved":
            ts = curved(src[j0:j1, 0:1], src[j0:j1, 1:2])
            tr = curved(rec[j0:j1, 0:1], rec[j0:j1, 1:2])
            return ts + tr, 1.0 / (ts * tr)
        ts, cs = _leg_time_and_cos(problem.velocity, src[j0:j1, 0:1], src[j0:j1, 1:2], pz, px, py)
        tr, cr = _leg_time_and_cos(problem.velocity, rec[j0:j1, 0:1], rec[j0:j1, 1:2], pz, px, py)
        return ts + tr, cs * cr / (ts * tr)

    wmax = torch.zeros(m, dtype=torch.float64, device=dev)
    for j0 in range(0, n, chunk):
        _, w = legs(j0, min(n, j0 + chunk))
        wmax = torch.maximum(wmax, w.max(dim=0).values)
    hw = int(math.ceil(half_width_s / dt))
    taps = torch.arange(-hw, hw + 1, device=dev, dtype=torch.int64)
    for j0 in range(0, n, chunk):
        j1 = min(n, j0 + chunk)
        tau, w = legs(j0, j1)
        amp = w / wmax[None, :]
        c = torch.round((tau - tf) / dt).to(torch.int64)  # nearest sample
        idx = c[..., None] + taps  # [nj, m, taps]
        t = tf + idx.to(torch.float64) * dt - tau[..., None]
        a = (math.pi * f_peak * t) ** 2
        val = amp[..., None] * (1.0 - 2.0 * a) * torch.exp(-a)
        ok = (idx >= 0) & (idx < nt)
        rows = torch.arange(j0, j1, device=dev, dtype=torch.int64)[:, None, None] * nt
        flat = (rows + idx)[ok]
        # overlapping wavelets: the deterministic (sorted) scatter keeps the
        # float32 sums, and so the samples, the same from run to run on a GPU
        was = torch.are_deterministic_algorithms_enabled()
        torch.use_deterministic_algorithms(True)
        try:
            out.index_add_(0, flat, val[ok].to(torch.float32))
        finally:
            torch.use_deterministic_algorithms(was)
    return out.view(n, nt)


def quantise(data: np.ndarray, kind: str):
    """Per-trace max-abs scaled 16-bit storage.

    sigma_j = max_i |D_j[i]| (1 where the trace is all zero); q = RNE(D / sigma_j)
    in bfloat16 or float16.  Returns (bits uint16 [n, n_t], sigma float32 [n],
    dequantised float64 [n, n_t] = q * sigma exactly)."""
    d = np.asarray(data, dtype=np.float32)
    sig = np.max(np.abs(d), axis=1).astype(np.float32)
    sig = np.where(sig > 0, sig, np.float32(1.0)).astype(np.float32)
    r = (d / sig[:, None]).astype(np.float32)
    if kind == "f16":
        q = r.astype(np.float16)
        bits = q.view(np.uint16)
        deq = q.astype(np.float64)
    elif kind == "bf16":
        b = r.view(np.uint32).astype(np.uint64)
        b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
        bits = b.astype(np.uint16)
        deq = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    else:
        raise ValueError(kind)
    return bits, sig, deq * sig.astype(np.float64)[:, None]


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def _finish(name, src, rec, n_t, dt, t_first, x, y, z, n_bins, dX, velocity, aperture_deg,
            weight=WEIGHT_COSCOS, **kw):
    src = np.asarray(src, dtype=np.float32)
    rec = np.asarray(rec, dtype=np.float32)
    bins = offset_bins(src, rec, dX, n_bins)
    src, rec, bins = _sort_by_bin(src, rec, bins)
    t0sq, s2 = traveltime_tables(z, velocity)
    r2 = aperture_table(t0sq, s2, aperture_deg)
    # The operator's model tables are float32 (the library's table type): the
    # FP64 reference checker and the kernels both take these rounded values.  r2 is rounded from
    # the FP64 tables (so that grid-aligned 45-degree ties stay exact).
    t0sq = t0sq.astype(np.float32).astype(np.float64)
    s2 = s2.astype(np.float32).astype(np.float64)
    return Problem(name=name, src=src, rec=rec, bin=bins, data=None, n_t=int(n_t), dt=float(dt),
                   t_first=float(t_first), x=np.asarray(x, np.float32), y=np.asarray(y, np.float32),
                   z=np.asarray(z, np.float64), n_bins=int(n_bins), t0sq=t0sq, s2=s2, r2=r2,
                   weight=weight, velocity=velocity, aperture_deg=aperture_deg,
                   offset_bin_width=float(dX), **kw)


def _pick_nodes(rng, ix_rng, iz_rng, n, min_sep_m, dx, dz, iy_rng=(0, 1), dy=1.0):
    nodes = []
    while len(nodes) < n:
        c = (int(rng.integers(*ix_rng)), int(rng.integers(*iy_rng)), int(rng.integers(*iz_rng)))
        ok = all(math.dist((c[0] * dx, c[1] * dy, c[2] * dz), (o[0] * dx, o[1] * dy, o[2] * dz)) >= min_sep_m
                 for o in nodes)
        if ok:
            nodes.append(c)
    return np.array(nodes, dtype=np.int64)


def make_line2d(seed=1):
    """2D constant-velocity split-spread line (v = 2000 m/s).

    32 shots at 50 m, 48 receivers per shot at 25 m (offsets (k - 23.5) * 25 m),
    500 samples at 4 ms; image 128 x 200 at 10 m (x = 140 + 10 i,
    z = 10 (k + 1)); 8 offset bins of 75 m; aperture 45 degrees; weight
    cos*cos/(Ts*Tr).  Data: 3 point diffractors at seeded grid nodes, 25 Hz
    Ricker, Gaussian noise with sigma = 1 % of the clean peak."""
    rng = np.random.default_rng(seed)
    sx = 50.0 * np.arange(32)
    h = (np.arange(48) - 23.5) * 25.0
    S, H = np.meshgrid(sx, h, indexing="ij")
    src = np.stack([S.ravel(), np.zeros(S.size)], 1)
    rec = np.stack([(S + H).ravel(), np.zeros(S.size)], 1)
    x = 140.0 + 10.0 * np.arange(128)
    z = 10.0 * (np.arange(200) + 1)
    p = _finish("line2d_const", src, rec, 500, 0.004, 0.0, x, [0.0], z, 8, 75.0, ("const", 2000.0), 45.0)
    nodes = _pick_nodes(rng, (30, 98), (30, 140), 3, 100.0, 10.0, 10.0)
    p.diffractor_nodes = nodes
    p.scatterers = np.stack([p.x[nodes[:, 0]].astype(np.float64), np.zeros(3), p.z[nodes[:, 2]]], 1)
    clean = model_scatterers(p, p.scatterers).numpy()
    sigma = 0.01 * float(np.max(np.abs(clean)))
    p.data = (clean + rng.normal(0.0, sigma, clean.shape)).astype(np.float32)
    p.meta["noise_sigma"] = sigma
    return p


def make_survey3d(seed=2, with_data=True, device=None, plane_spacing=250.0):
    """3D v(z) survey: v = 1500 + 0.5 z, straight-ray RMS traveltimes.

    10 x 10 shots at 500 m (250 .. 4750 m); each shot records a 40 x 50
    receiver patch at 25 m (offsets ((a - 19.5) 25, (b - 24.5) 25)), giving
    200 000 traces of 1500 samples at 4 ms.  Image 256 x 256 x 400 at
    12.5 / 12.5 / 5 m centred on (2500, 2500), 16 offset bins of 50 m,
    aperture 60 degrees.  Data: 20 seeded diffractors (z 200-1800 m) and 3
    seeded dipping planes (z0 in [400, 1600] m, dip <= 20 deg) represented by
    point scatterers on a `plane_spacing` grid; 25 Hz Ricker; no noise."""
    rng = np.random.default_rng(seed)
    s1 = 250.0 + 500.0 * np.arange(10)
    SX, SY = np.meshgrid(s1, s1, indexing="ij")
    a = (np.arange(40) - 19.5) * 25.0
    b = (np.arange(50) - 24.5) * 25.0
    HA, HB = np.meshgrid(a, b, indexing="ij")
    sx = np.repeat(SX.ravel(), HA.size)
    sy = np.repeat(SY.ravel(), HA.size)
    rx = sx + np.tile(HA.ravel(), SX.size)
    ry = sy + np.tile(HB.ravel(), SX.size)
    x = 2500.0 + (np.arange(256) - 127.5) * 12.5
    z = 5.0 * (np.arange(400) + 1)
    p = _finish("survey3d_vz", np.stack([sx, sy], 1), np.stack([rx, ry], 1), 1500, 0.004, 0.0, x, x.copy(), z,
                16, 50.0, ("linear", 1500.0, 0.5), 60.0)
    nodes = _pick_nodes(rng, (16, 240), (39, 360), 20, 100.0, 12.5, 5.0, iy_rng=(16, 240), dy=12.5)
    p.diffractor_nodes = nodes
    diff = np.stack([p.x[nodes[:, 0]], p.y[nodes[:, 1]], p.z[nodes[:, 2]]], 1).astype(np.float64)
    g = np.arange(0.0, 5000.0 + 1e-9, plane_spacing)
    GX, GY = np.meshgrid(g, g, indexing="ij")
    planes = []
    for _ in range(3):
        z0 = rng.uniform(400.0, 1600.0)
        dip = math.radians(rng.uniform(0.0, 20.0))
        az = rng.uniform(0.0, 2 * math.pi)
        px_, py_ = math.tan(dip) * math.cos(az), math.tan(dip) * math.sin(az)
        zz = z0 + px_ * (GX - 2500.0) + py_ * (GY - 2500.0)
        planes.append(np.stack([GX.ravel(), GY.ravel(), zz.ravel()], 1))
    p.scatterers = np.concatenate([diff] + planes, 0)
    if with_data:
        p.data = model_scatterers(p, p.scatterers, device=device)
        if device is None:
            p.data = p.data.numpy()
    return p


def make_line2d_vz(seed=4, n_shots=256, n_rec=240, n_t=2000, nx=1024, nz=800, n_bins=32):
    """2D v(z) line for the adjoint pair: v = 1500 + 0.5 z (RMS traveltimes).

    256 shots at 37.5 m; 240 split-spread receivers at 12.5 m (offsets
    (k - 119.5) * 12.5 m); 2000 samples at 4 ms; image 1024 at 10 m centred on
    the line, z = 5 (k + 1) (800 depths); 32 offset bins of 46.875 m;
    aperture 60 degrees.  Data are not set (the adjoint checks use N(0, 1)
    vectors; least squares uses demigrated spikes)."""
    s = 37.5 * np.arange(n_shots)
    h = (np.arange(n_rec) - (n_rec - 1) / 2.0) * 12.5
    S, H = np.meshgrid(s, h, indexing="ij")
    src = np.stack([S.ravel(), np.zeros(S.size)], 1)
    rec = np.stack([(S + H).ravel(), np.zeros(S.size)], 1)
    xc = 0.5 * (s[0] + s[-1])
    x = xc + (np.arange(nx) - (nx - 1) / 2.0) * 10.0
    z = 5.0 * (np.arange(nz) + 1)
    dX = (np.max(np.abs(h)) + 6.25) / n_bins
    return _finish("line2d_vz", src, rec, n_t, 0.004, 0.0, x, [0.0], z, n_bins, dX,
                   ("linear", 1500.0, 0.5), 60.0)


def bin_offsets(problem: Problem) -> np.ndarray:
    """Mean absolute offset |x_s - x_r| of the traces of each bin (FP64; the
    bin's lower edge midpoint when it holds no trace)."""
    h = np.hypot(problem.src[:, 0].astype(np.float64) - problem.rec[:, 0],
                 problem.src[:, 1].astype(np.float64) - problem.rec[:, 1])
    out = np.zeros(problem.n_bins)
    width = problem.offset_bin_width or 1.0
    for b in range(problem.n_bins):
        sel = problem.bin == b
        out[b] = h[sel].mean() if sel.any() else (b + 0.5) * width
    return out


def make_flat_line(v_true=2000.0, v_mig=2000.0, z_reflector=800.0, n_t=400, nz=240, nx=5, n_bins=10,
                   bin_width=100.0, f_peak=25.0):
    """2D line over one flat reflector in a constant-velocity earth, for the
    moveout measure of the offset images.

    Shots every 50 m over 0 .. 4000 m, split-spread receivers every 50 m with
    offsets -1000 .. 1000 m; 400 samples at 4 ms.  Each trace holds the
    reflection of the flat interface at z_reflector computed with v_true: a
    25 Hz Ricker at t = 2 sqrt(z^2 + (h/2)^2) / v_true, unit amplitude.  The
    traveltime tables are those of v_mig (so v_mig != v_true is a velocity
    error).  Image: nx columns at 50 m around x = 2000 m, z = 5 (k + 1) m,
    n_bins bins of |h| of bin_width m, aperture 60 degrees."""
    s = 50.0 * np.arange(81)
    h = 50.0 * (np.arange(41) - 20)
    S, H = np.meshgrid(s, h, indexing="ij")
    src = np.stack([S.ravel(), np.zeros(S.size)], 1)
    rec = np.stack([(S + H).ravel(), np.zeros(S.size)], 1)
    x = 2000.0 + 50.0 * (np.arange(nx) - (nx - 1) / 2.0)
    z = 5.0 * (np.arange(nz) + 1)
    p = _finish("flat_line", src, rec, n_t, 0.004, 0.0, x, [0.0], z, n_bins, bin_width, ("const", v_mig), 60.0)
    hh = np.abs(p.src[:, 0].astype(np.float64) - p.rec[:, 0])
    t_ref = 2.0 * np.sqrt(z_reflector ** 2 + 0.25 * hh * hh) / v_true
    t = np.arange(n_t) * p.dt
    p.data = ricker(t[None, :] - t_ref[:, None], f_peak).astype(np.float32)
    p.meta = dict(v_true=v_true, v_mig=v_mig, z_reflector=z_reflector)
    return p


def rho_filter_taps(dt: float, alpha: float = 0.5, half_len: int = 32, n_fft: int = 8192):
    """Taps (float32 [2 half_len + 1], centre index half_len) of the
    anti-causal fractional derivative (-i w)^alpha in numpy's e^{+i w t}
    convention (alpha = 1 is -d/dt), by frequency sampling on n_fft points and
    a Hann window.  Summing a trace family along a traveltime surface that
    only lies later than its apex acts on the wavelet as (-i w)^(-1/2) per
    summed surface dimension, so alpha = 1/2 restores a zero-phase image for a
    line (2D) and alpha = 1 for an areal (3D) acquisition."""
    w = 2.0 * math.pi * np.fft.fftfreq(n_fft, dt)
    H = np.power(-1j * w, alpha)
    h = np.real(np.fft.ifft(H))
    M = int(half_len)
    taps = np.concatenate([h[n_fft - M:], h[:M + 1]])
    win = 0.5 * (1.0 + np.cos(math.pi * np.arange(-M, M + 1) / (M + 1)))
    return (taps * win).astype(np.float32), M


def make_diffractor_line(v=2000.0, x_diff=1000.0, z_diff=600.0, spacing=5.0, n_t=400, dz=2.0, nz=400):
    """2D zero-offset line over one point diffractor in a constant-velocity
    earth (no noise): coincident source and receiver every `spacing` m over
    0 .. 2000 m, 400 samples at 4 ms, 25 Hz Ricker with the cos cos / (T T)
    amplitude; image: the single column at x_diff, z = dz (k + 1), one bin,
    aperture 60 degrees."""
    s = np.arange(0.0, 2000.0 + 1e-9, spacing)
    src = np.stack([s, np.zeros(s.size)], 1)
    z = dz * (np.arange(nz) + 1)
    p = _finish("diffractor_line", src, src.copy(), n_t, 0.004, 0.0, [x_diff], [0.0], z, 1, 1e9,
                ("const", v), 60.0)
    p.scatterers = np.array([[x_diff, 0.0, z_diff]])
    p.data = model_scatterers(p, p.scatterers).numpy()
    return p


def batch_line_shapes(seed=5, n_lines=64):
    """Shapes of the uneven batch: (n_shots, n_rec, n_t, nx, nz) per line,
    drawn inclusive from U{16..512}, U{48..480}, U{1000..3000}, U{256..2048},
    U{400..1000}."""
    rng = np.random.default_rng(seed)
    return [tuple(int(v) for v in (rng.integers(16, 513), rng.integers(48, 481), rng.integers(1000, 3001),
                                   rng.integers(256, 2049), rng.integers(400, 1001)))
            for _ in range(n_lines)]


def make_batch_line(shape, index=0):
    """One line of the uneven batch: shots at 25 m, split-spread receivers at
    12.5 m, image dx 12.5 m centred, dz 5 m, dt 4 ms, v = 1500 + 0.5 z,
    16 offset bins of max|h| / 16, aperture 60 degrees.  Data not set."""
    ns, nr, nt, nx, nz = shape
    s = 25.0 * np.arange(ns)
    h = (np.arange(nr) - (nr - 1) / 2.0) * 12.5
    S, H = np.meshgrid(s, h, indexing="ij")
    src = np.stack([S.ravel(), np.zeros(S.size)], 1)
    rec = np.stack([(S + H).ravel(), np.zeros(S.size)], 1)
    xc = 0.5 * (s[0] + s[-1])
    x = xc + (np.arange(nx) - (nx - 1) / 2.0) * 12.5
    z = 5.0 * (np.arange(nz) + 1)
    hmax = float(np.max(np.abs(h)))
    dX = hmax / 16.0 * (1.0 + 1e-9)
    return _finish(f"batch_line_{index}", src, rec, nt, 0.004, 0.0, x, [0.0], z, 16, dX,
                   ("linear", 1500.0, 0.5), 60.0)


def with_diffractors(p: Problem, seed: int, n: int = 3, min_sep_m: float = 100.0, device=None) -> Problem:
    """Point diffractors at seeded image grid nodes of a 2D line (the middle
    half of its columns and of its depths, at least min_sep_m apart); the
    traces become their modelled data (25 Hz Ricker, no noise)."""
    rng = np.random.default_rng(seed)
    nx, nz = len(p.x), len(p.z)
    dx = float(p.x[1] - p.x[0]) if nx > 1 else 1.0
    dz = float(p.z[1] - p.z[0]) if nz > 1 else 1.0
    nodes = _pick_nodes(rng, (nx // 4, max(nx // 4 + 1, 3 * nx // 4)), (nz // 4, max(nz // 4 + 1, 3 * nz // 4)), n,
                        min_sep_m, dx, dz)
    p.diffractor_nodes = nodes
    p.scatterers = np.stack([p.x[nodes[:, 0]].astype(np.float64), np.zeros(n), p.z[nodes[:, 2]]], 1)
    p.data = model_scatterers(p, p.scatterers, device=device).cpu().numpy()
    return p


def make_random(seed, n_traces, n_t, nx, ny, nz, n_bins, velocity=("linear", 1500.0, 0.5),
                aperture_deg=60.0, dx=12.5, dz=5.0, spread=600.0, t_first=0.0, dt=0.004,
                weight=WEIGHT_COSCOS, data="bandlimited"):
    """Small random problem for parity and invariant tests: sources and
    receivers uniformly scattered around the image area.  data="bandlimited"
    (default): Gaussian noise filtered by a 25 Hz Ricker wavelet and scaled to
    unit RMS, i.e. seismic-like band-limited traces; data="normal": white
    N(0, 1) samples (a stress case for time rounding); None: no data."""
    rng = np.random.default_rng(seed)
    x = (np.arange(nx) - (nx - 1) / 2.0) * dx + 1000.0
    y = ((np.arange(ny) - (ny - 1) / 2.0) * dx + 2000.0) if ny > 1 else np.array([0.0])
    cx, cy = 1000.0, (2000.0 if ny > 1 else 0.0)
    half_x = 0.5 * nx * dx + spread
    half_y = (0.5 * ny * dx + spread) if ny > 1 else 0.0
    src = np.stack([rng.uniform(cx - half_x, cx + half_x, n_traces),
                    rng.uniform(cy - half_y, cy + half_y, n_traces)], 1)
    rec = np.stack([rng.uniform(cx - half_x, cx + half_x, n_traces),
                    rng.uniform(cy - half_y, cy + half_y, n_traces)], 1)
    if ny == 1:
        src[:, 1] = 0.0
        rec[:, 1] = 0.0
    z = dz * (np.arange(nz) + 1)
    hmax = float(np.max(np.hypot(src[:, 0] - rec[:, 0], src[:, 1] - rec[:, 1]))) if n_traces else 1.0
    dX = max(hmax, 1.0) / n_bins * (1.0 + 1e-9)
    p = _finish(f"random_{seed}", src, rec, n_t, dt, t_first, x, y, z, n_bins, dX, velocity, aperture_deg,
                weight=weight)
    if data == "normal":
        p.data = rng.standard_normal((p.n_traces, n_t)).astype(np.float32)
    elif data == "bandlimited":
        p.data = bandlimited_noise(rng, p.n_traces, n_t, dt)
    return p


def bandlimited_noise(rng, n_traces: int, n_t: int, dt: float, f_peak: float = 25.0) -> np.ndarray:
    """Gaussian noise convolved with a Ricker wavelet (zero phase), unit RMS, float32."""
    w = ricker(np.arange(-int(0.08 / dt), int(0.08 / dt) + 1) * dt, f_peak)
    raw = rng.standard_normal((n_traces, n_t + len(w) - 1))
    out = np.zeros((n_traces, n_t))
    for k, c in enumerate(w):
        out += c * raw[:, k:k + n_t]
    rms = float(np.sqrt(np.mean(out * out))) if out.size else 1.0
    return (out / (rms if rms > 0 else 1.0)).astype(np.float32)


def random_image(problem: Problem, seed: int) -> np.ndarray:
    """N(0, 1) float32 image of the problem's shape."""
    return np.random.default_rng(seed).standard_normal(problem.image_shape).astype(np.float32)


def bandlimited_image(problem: Problem, seed: int) -> np.ndarray:
    """N(0, 1) image smoothed along depth by a Ricker wavelet (a reflectivity-
    like, band-limited image), unit RMS, float32."""
    rng = np.random.default_rng(seed)
    nb, ny, nx, nz = problem.image_shape
    flat = bandlimited_noise(rng, nb * ny * nx, nz, 0.004)
    return flat.reshape(nb, ny, nx, nz)


def random_data(problem: Problem, seed: int) -> np.ndarray:
    """N(0, 1) float32 traces of the problem's shape."""
    return np.random.default_rng(seed).standard_normal((problem.n_traces, problem.n_t)).astype(np.float32)
