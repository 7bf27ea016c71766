"""FP64 CPU oracle for the offset stack and the common-image-gather moveout
measure.

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark's CPU
baseline, never by the GPU library or its binding.

What it computes (Introduction): migration of redundant data gives one image
per offset bin; the depth at which the same reflector appears in different
offset images measures the error of the velocity model, and once the images
agree they are added into one stacked image.  Made concrete here:

* stack      S[y][x][z] = sum over bins b of I[b][y][x][z].
* moveout    for every image column and bin, the depth displacement of the
             bin's image against the stack over a depth window [z_lo, z_hi):
                 C_b(l) = sum_{z in window} S[z] * I_b[z + l],  l = -L..L,
             with I_b = 0 outside [0, nz).  l* maximises C_b; ties go to the
             smaller |l|, then to the negative l.  When |l*| < L and the
             parabola through C_b(l*-1), C_b(l*), C_b(l*+1) opens downwards,
             the vertex refines it:
                 shift = l* + (C(l*-1) - C(l*+1)) / (2 (C(l*-1) - 2 C(l*) + C(l*+1)))
             else shift = l*.  shift > 0: the bin images the event deeper
             than the stack, in depth samples.  peak = C_b(l*).
* curvature  per column, the least-squares slope of shift_b against h_b^2
             (h_b = the bin's centre offset) over the bins with peak > 0;
             0 when fewer than two such bins or all h_b^2 are equal.
             Units: depth samples per m^2.  A velocity that is too low images
             a flat reflector shallower at larger offsets (negative slope).

Parity status: pinned by the CPU tests (stack = the migration of all traces
in one bin; exact zero shift for identical gathers; recovered shifts of
displaced wavelets; the flat-reflector residual moveout of a constant
velocity error against its closed form).
"""
from __future__ import annotations

import numpy as np


def stack(image: np.ndarray) -> np.ndarray:
    """Sum of the offset images: image [n_bins, ...] -> [...] (float64)."""
    return np.asarray(image, dtype=np.float64).sum(axis=0)


def _lag_order(max_lag: int) -> list[int]:
    order = [0]
    for m in range(1, max_lag + 1):
        order += [-m, m]
    return order


def correlations(image: np.ndarray, max_lag: int, z_lo: int = 0, z_hi: int | None = None) -> np.ndarray:
    """C[b, y, x, l + L] = sum_{z_lo <= z < z_hi} S[y, x, z] * I[b, y, x, z + l] (FP64)."""
    img = np.asarray(image, dtype=np.float64)
    nb, ny, nx, nz = img.shape
    z_hi = nz if z_hi is None else z_hi
    s = img.sum(axis=0)[..., z_lo:z_hi]
    L = max_lag
    padded = np.zeros((nb, ny, nx, nz + 2 * L))
    padded[..., L:L + nz] = img
    out = np.empty((nb, ny, nx, 2 * L + 1))
    for j, lag in enumerate(range(-L, L + 1)):
        seg = padded[..., L + z_lo + lag:L + z_hi + lag]
        out[..., j] = np.einsum("yxz,byxz->byx", s, seg)
    return out


def cig_moveout(image: np.ndarray, offsets: np.ndarray, max_lag: int, z_lo: int = 0, z_hi: int | None = None):
    """(stack, shift, peak, curvature) of the offset images [n_bins, ny, nx, nz]."""
    img = np.asarray(image, dtype=np.float64)
    nb, ny, nx, nz = img.shape
    C = correlations(img, max_lag, z_lo, z_hi)
    L = max_lag
    shift = np.zeros((nb, ny, nx))
    peak = np.zeros((nb, ny, nx))
    order = _lag_order(L)
    for b in range(nb):
        for iy in range(ny):
            for ix in range(nx):
                c = C[b, iy, ix]
                best = order[0]
                for lag in order[1:]:
                    if c[lag + L] > c[best + L]:
                        best = lag
                s = float(best)
                if abs(best) < L:
                    cm, c0, cp = c[best + L - 1], c[best + L], c[best + L + 1]
                    den = cm - 2.0 * c0 + cp
                    if den < 0.0:
                        s = best + 0.5 * (cm - cp) / den
                shift[b, iy, ix] = s
                peak[b, iy, ix] = c[best + L]
    q = np.asarray(offsets, dtype=np.float64) ** 2
    curv = np.zeros((ny, nx))
    for iy in range(ny):
        for ix in range(nx):
            use = peak[:, iy, ix] > 0.0
            if use.sum() < 2:
                continue
            qq = q[use]
            ss = shift[use, iy, ix]
            dq = qq - qq.mean()
            den = float((dq * dq).sum())
            if den > 0.0:
                curv[iy, ix] = float((dq * (ss - ss.mean())).sum()) / den
    return img.sum(axis=0), shift, peak, curv


def flat_reflector_depth(z_true: float, h: float, v_true: float, v_mig: float) -> float:
    """Depth at which constant-velocity migration with v_mig images a flat
    reflector at z_true (true velocity v_true) from a source-receiver pair of
    offset h, at the common midpoint: the two-way time 2 sqrt(z^2 + h^2 / 4) / v
    is matched with the migration velocity."""
    t = 2.0 * np.sqrt(z_true ** 2 + 0.25 * h * h) / v_true
    return float(np.sqrt(max((0.5 * v_mig * t) ** 2 - 0.25 * h * h, 0.0)))
