"""LoRADS, Algorithm 2: Phase I (LRALM) -> switch -> Phase II (LRADMM).

Switch (Section 4.1 and the heuristic factor of Section 5.1): U0 = V0 = the
Phase-I factor, the multiplier carried over (the oracle's Phase I already uses
the X-multiplier, which is half the multiplier of the factored system), and
rho multiplied by h.  Output: U_hat = (U + V)/2, X_hat = U_hat U_hat^T.
"""
from __future__ import annotations

import numpy as np

from . import admm as admm_mod
from . import alm as alm_mod
from . import metrics


def lorads(prob, U0, opts, lam0=None, with_metrics=True, progress=None):
    lam0 = np.zeros(prob.m) if lam0 is None else np.asarray(lam0, dtype=np.float64)
    if opts.phase1:
        p1 = alm_mod.alm(prob, U0, lam0, opts, progress=progress)
        U, lam, rho = p1["U"], p1["lam"], p1["rho"]
    else:
        p1 = None
        U, lam = np.asarray(U0, dtype=np.float64), lam0
        rho = opts.rho0 if opts.rho0 > 0 else 1.0 / max(1.0, float(np.max(np.abs(prob.b))))
    rho_admm = opts.h * rho
    p2 = admm_mod.admm(prob, U, U, lam, rho_admm, opts, progress=progress)
    Uh = 0.5 * (p2["U"] + p2["V"])
    out = dict(phase1=p1, phase2=p2, U_hat=Uh, lam=p2["lam"], rank=Uh.shape[1])
    if with_metrics:
        out["metrics"] = metrics.appendix_b(prob, Uh, p2["lam"])
    return out
