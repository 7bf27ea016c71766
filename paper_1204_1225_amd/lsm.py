"""Least-squares migration by steepest descent with exact line search.

Objective J(m) = 1/2 ||L m - d||^2 with L = demigration (Kirchhoff modelling)
and L^T = migration.  Each step: g = L^T r (migrate the residual), q = L g
(demigrate), alpha = ||g||^2 / ||q||^2, m -= alpha g, r -= alpha q.  For a
quadratic J this step is the exact minimiser along -g and decreases J by
||g||^4 / (2 ||q||^2).  The scalars are float64 device reductions of the
library (km_dot_f64); only they cross to the host, and the updates are the
library's axpby kernel.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import torch

from . import ops


@dataclasses.dataclass
class LsmResult:
    image: torch.Tensor
    objective: List[float]        # J before step 0 and after every step
    predicted_decrease: List[float]  # ||g||^4 / (2 ||Lg||^2) per step
    steps: int


def lsm(dp: "ops.DeviceProblem", d_obs: torch.Tensor, n_iter: int = 10, m0: Optional[torch.Tensor] = None,
        checkpoint: Optional[str] = None) -> LsmResult:
    """Run n_iter steps from m0 (default zero image).  If `checkpoint` is a
    path, (m, r, history, k) is saved after every step with torch.save and a
    run started with an existing checkpoint resumes from it."""
    dev = dp.device
    start = 0
    obj: List[float] = []
    pred: List[float] = []
    if checkpoint is not None:
        import os

        if os.path.exists(checkpoint):
            st = torch.load(checkpoint, map_location=dev, weights_only=True)
            m, r = st["m"], st["r"]
            obj, pred, start = list(st["objective"]), list(st["predicted"]), int(st["k"])
    if start == 0:
        m = torch.zeros(dp.image_shape, dtype=torch.float32, device=dev) if m0 is None else m0.clone()
        # r = L m - d
        r = torch.empty((dp.n_traces, dp.n_t), dtype=torch.float32, device=dev)
        ops.axpby(-1.0, d_obs.contiguous(), 0.0, r)
        if m0 is not None:
            ops.demigrate(dp, m, out=r, accumulate=True)
        obj = [0.5 * float(ops.dot_f64(r, r))]
    g = torch.empty_like(m)
    q = torch.empty_like(r)
    for k in range(start, n_iter):
        ops.migrate(dp, data=r, image=g, dtype="f32")
        ops.demigrate(dp, g, out=q)
        gg = float(ops.dot_f64(g, g))
        qq = float(ops.dot_f64(q, q))
        if qq == 0.0 or gg == 0.0:
            break
        alpha = gg / qq
        ops.axpby(-alpha, g, 1.0, m)
        ops.axpby(-alpha, q, 1.0, r)
        obj.append(0.5 * float(ops.dot_f64(r, r)))
        pred.append(gg * gg / (2.0 * qq))
        if checkpoint is not None:
            torch.save({"m": m, "r": r, "objective": obj, "predicted": pred, "k": k + 1}, checkpoint)
    return LsmResult(image=m, objective=obj, predicted_decrease=pred, steps=len(obj) - 1)
