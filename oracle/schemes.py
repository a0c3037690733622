"""The two IMPES schemes (oracle; test infrastructure).

Alg. 1 (high-dimensional scheme): per step the fine pressure (Def.
pressureDG with the mobility of s^n), the velocity (Def. velocityDG), the
saturation (Def. saturationDG) and the limiter (eq. limiterMain).
Alg. 3 (LRBMS scheme), step 5: the online step of ``online.online_step``.
The initial projection of s0 is trivial for s0 = 0 (every configuration).
"""
from __future__ import annotations

import numpy as np

from .pressure import Mobility, fine_pressure, reconstruct_flux
from .transport import saturation_step
from .online import online_step, DIRECT


def fine_impes(grid, prob, s0, n_steps, callback=None):
    s = s0.copy()
    hist = []
    for n in range(n_steps):
        p = fine_pressure(grid, prob, s=s)
        F = reconstruct_flux(grid, prob, p, Mobility(grid, prob, s=s))
        s, flags = saturation_step(grid, prob, s, F)
        hist.append(dict(p=p, F=F, s=s.copy(), flags=flags))
        if callback:
            callback(n, hist[-1])
    return s, hist


def lrbms_impes(model, s0, n_steps, mode=DIRECT, callback=None):
    s = s0.copy()
    hist = []
    for n in range(n_steps):
        out = online_step(model, s, mode)
        s = out["s"]
        hist.append(out)
        if callback:
            callback(n, out)
    return s, hist
