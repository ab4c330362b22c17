"""LRADMM (Algorithm 1) on the penalised split problem, linear objective.

Augmented Lagrangian, eq. (ALF):
    L_rho(U, V, lam) = <C, U V^T> + gamma/2 ||U - V||_F^2
                       + lam^T (A(U V^T) - b) + rho/2 ||A(U V^T) - b||^2.

One iteration:
  U^{k+1} = argmin_U L_rho(U, V^k, lam^k)     -- linear system (linU)
  V^{k+1} = argmin_V L_rho(U^{k+1}, V, lam^k) -- linear system (linV)
  lam^{k+1} = lam^k + rho (A(U^{k+1} V^{k+1 T}) - b)

Both systems are solved by CG warm-started at the other factor (Section 4.4):
with W the fixed factor and x = W + D, the residual at x0 = W is
    R0 = -(C + A*(lam + rho (A(W W^T) - b))) W,
the negative gradient of L_rho in the free factor at W, so CG solves M_W D = R0.

With the quadratic objective f(X) = <C, X> + (mu/2) ||X||_F^2 (Section 1's
convex f), grad f(U W^T) W = C W + mu U (W^T W) is still linear in the free
factor, so both subproblems stay linear systems: the operator gains
mu P (W^T W) and R0 the term -mu W (W^T W).

Stop, eq. (stop): max{ ||A(U V^T) - b||_2 / (1 + ||b||_inf),
                       gamma ||V^{k+1} - V^k||_F / (1 + ||V^k||_F) } < eps.
rho schedule (Section 5.1): every 5th iteration rho <- min(1.2 rho, rho_max),
never decreased.  gamma: the rule of `Options.gamma` (the paper leaves it open).
"""
from __future__ import annotations

import math

import numpy as np

from . import operators
from .cg import cg, cg_operator


def grad_factor(prob, W, lam, rho):
    """(C + A*(lam + rho (A(W W^T) - b))) W, the gradient of L_rho in the free
    factor evaluated at the fixed factor W (both factors equal W)."""
    z = operators.forward(prob, W, W)
    w = lam + rho * (z - prob.b)
    g = operators.adjoint(prob, w, 1.0, W)
    mu = operators.mu_of(prob)
    if mu != 0.0:
        g = g + mu * (W @ (W.T @ W))
    return g


def alf(prob, U, V, lam, rho, gamma):
    """eq. (ALF) with f(X) = <C, X> + (mu/2) ||X||_F^2."""
    z = operators.forward(prob, U, V) - prob.b
    return (operators.objective(prob, U, V) + 0.5 * gamma * float(np.sum((U - V) ** 2))
            + float(lam @ z) + 0.5 * rho * float(z @ z))


def cg_tolerance(opts, kkt_prev: float) -> float:
    return min(opts.cg_tol_max, max(opts.cg_tol_floor, opts.cg_tol_kkt * kkt_prev))


def half_step(prob, W, lam, rho, gamma, tol, maxit):
    """argmin over the free factor with the other factor fixed at W, by CG from
    x0 = W.  Returns (new factor, CG iterations)."""
    R0 = -grad_factor(prob, W, lam, rho)
    D, it, _, _ = cg(cg_operator(prob, W, rho, gamma), R0, tol, maxit)
    return W + D, it


def admm(prob, U0, V0, lam0, rho0, opts, trace=None, progress=None):
    """progress (optional): called with a status line every 100 iterations."""
    U = np.array(U0, dtype=np.float64)
    V = np.array(V0, dtype=np.float64)
    lam = np.array(lam0, dtype=np.float64)
    rho = float(rho0)
    n, r = V.shape
    nrm = operators.norms(prob)
    maxit = min(n * r, opts.cg_maxit)
    kkt = math.inf
    cg_total = 0
    k = 0
    pinf = dres = math.inf
    c_norm2 = operators.cost_norm2(prob) if (opts.gamma_rule == 1 and opts.gamma_fixed <= 0) else None
    while k < opts.max_admm_iter:
        gamma = opts.gamma(nrm["c_fro"], n, c_norm2)
        tol = cg_tolerance(opts, kkt)
        U, it_u = half_step(prob, V, lam, rho, gamma, tol, maxit)
        V_new, it_v = half_step(prob, U, lam, rho, gamma, tol, maxit)
        z = operators.forward(prob, U, V_new) - prob.b
        lam_new = lam + rho * z
        pinf = float(np.linalg.norm(z)) / (1.0 + nrm["b_inf"])
        dres = gamma * float(np.linalg.norm(V_new - V)) / (1.0 + float(np.linalg.norm(V)))
        if trace is not None:
            trace.append(dict(k=k, U=U.copy(), V_old=V.copy(), V=V_new.copy(), lam_old=lam.copy(),
                              lam=lam_new.copy(), rho=rho, gamma=gamma, cg=(it_u, it_v),
                              pinf=pinf, dres=dres))
        kkt = max(pinf, dres)
        V = V_new
        lam = lam_new
        cg_total += it_u + it_v
        k += 1
        if progress is not None and k % 100 == 0:
            progress(f"ADMM {k}: eq. (stop) {kkt:.3e}")
        if kkt < opts.eps:
            break
        if k % opts.rho_every == 0 and rho < opts.rho_max:
            rho = min(opts.rho_growth * rho, opts.rho_max)
    return dict(U=U, V=V, lam=lam, rho=rho, iters=k, cg_iters=cg_total, kkt=kkt,
                pinf=pinf, dres=dres, converged=kkt < opts.eps)
