"""LRALM: the Burer-Monteiro augmented Lagrangian warm start (Phase I).

Section 4.1: Phase I applies the augmented Lagrangian method of Burer and
Monteiro to the factorised problem (BM), min <C, U U^T> s.t. A(U U^T) = b,
from a random start with L-BFGS as the inner solver.  Section 4.3 and 5.1 add
the dynamic rank: start at a logarithmic rank and multiply it by 1.5 whenever
an inner solve is judged hard by its iteration count.

The oracle works with the multiplier lam of the constraint A(X) = b written on
X = U U^T (the X-multiplier; it equals half the multiplier of the factored
KKT system, which is why Algorithm 2 hands lam/2 of that system to ADMM):

    L(U) = <C, U U^T> + lam^T (A(U U^T) - b) + rho/2 ||A(U U^T) - b||^2,
    grad L(U) = 2 (C + A*(lam + rho (A(U U^T) - b))) U.

Exact line search: L(U + a D) is a quartic in a because U U^T moves along
U U^T + a (U D^T + D U^T) + a^2 D D^T; its coefficients need A(U D^T), A(D D^T),
<C D, U> and <C D, D>, and the step is the minimiser among the positive real
roots of the cubic derivative.

With the quadratic objective f(X) = <C, X> + (mu/2) ||X||_F^2 (Section 1's
convex f) the same holds with <C, U U^T> replaced by f(U U^T): the gradient
gains 2 mu U (U^T U), and ||(U + a D)(U + a D)^T||_F^2 = ||A0 + a A1 + a^2 A2||_F^2
with A0 = U^T U, A1 = U^T D + D^T U, A2 = D^T D adds to every coefficient of the
quartic.

The inner and outer rules, tolerances and rank-growth trigger are the readings
documented in `oracle/options.py`.
"""
from __future__ import annotations

import math

import numpy as np

from . import operators, rng


def objective_parts(prob, U, lam, rho):
    z = operators.forward(prob, U, U) - prob.b
    return operators.objective(prob, U, U) + float(lam @ z) + 0.5 * rho * float(z @ z)


def gradient(prob, U, z, lam, rho):
    w = lam + rho * (z - prob.b)
    g = 2.0 * operators.adjoint(prob, w, 1.0, U)
    mu = operators.mu_of(prob)
    if mu != 0.0:
        g = g + 2.0 * mu * (U @ (U.T @ U))
    return g


def quartic_coefficients(prob, U, D, z, lam, rho):
    """Coefficients (q1, q2, q3, q4) of L(U + a D) - L(U) = q1 a + q2 a^2 +
    q3 a^3 + q4 a^4."""
    p0 = z - prob.b
    p1 = 2.0 * operators.forward(prob, U, D)
    p2 = operators.forward(prob, D, D)
    CD = operators.cost_apply(prob, D)
    c1 = 2.0 * float(np.sum(CD * U))
    c2 = float(np.sum(CD * D))
    q4 = 0.5 * rho * float(p2 @ p2)
    q3 = rho * float(p1 @ p2)
    q2 = c2 + float(lam @ p2) + 0.5 * rho * (float(p1 @ p1) + 2.0 * float(p0 @ p2))
    q1 = c1 + float(lam @ p1) + rho * float(p0 @ p1)
    mu = operators.mu_of(prob)
    if mu != 0.0:
        A0, A2 = U.T @ U, D.T @ D
        A1 = U.T @ D + D.T @ U
        ip = lambda X, Y: float(np.sum(X * Y))
        q1 += mu * ip(A0, A1)
        q2 += 0.5 * mu * (ip(A1, A1) + 2.0 * ip(A0, A2))
        q3 += mu * ip(A1, A2)
        q4 += 0.5 * mu * ip(A2, A2)
    return q1, q2, q3, q4


def quartic_step(q1, q2, q3, q4):
    """Minimiser of phi(a) = q1 a + q2 a^2 + q3 a^3 + q4 a^4 over a > 0, taken
    among the real roots of phi'(a) = q1 + 2 q2 a + 3 q3 a^2 + 4 q4 a^3."""
    coeffs = [4.0 * q4, 3.0 * q3, 2.0 * q2, q1]
    while len(coeffs) > 1 and coeffs[0] == 0.0:
        coeffs = coeffs[1:]
    if len(coeffs) == 1:
        return 0.0
    roots = np.roots(coeffs)
    best, best_val = 0.0, 0.0
    for z in roots:
        if abs(z.imag) > 1e-8 * max(1.0, abs(z.real)):
            continue
        a = float(z.real)
        if a <= 0.0:
            continue
        val = ((q4 * a + q3) * a + q2) * a * a + q1 * a
        if val < best_val:
            best, best_val = a, val
    return best


def grow_rank(U, r_new, event, seed):
    n, r = U.shape
    sigma = 1e-3 * float(np.linalg.norm(U)) / math.sqrt(n * r)
    extra = sigma * rng.normals(seed, event, n * (r_new - r)).reshape(n, r_new - r)
    return np.hstack([U, extra])


def lbfgs_inner(prob, U, lam, rho, tol, cap, mem, c_fro):
    """Minimise L(U) by L-BFGS with exact line search.  Returns (U, z, iters,
    converged)."""
    z = operators.forward(prob, U, U)
    G = gradient(prob, U, z, lam, rho)
    hist = []
    it = 0
    while True:
        gnorm = float(np.linalg.norm(G))
        if gnorm / (1.0 + c_fro) <= tol:
            return U, z, it, True
        if it >= cap:
            return U, z, it, False
        # two-loop recursion
        q = G.copy()
        alphas = []
        for S, Y, rh in reversed(hist):
            a = rh * float(np.sum(S * q))
            q -= a * Y
            alphas.append(a)
        if hist:
            S, Y, _ = hist[-1]
            q *= float(np.sum(S * Y)) / float(np.sum(Y * Y))
        for (S, Y, rh), a in zip(hist, reversed(alphas)):
            bt = rh * float(np.sum(Y * q))
            q += (a - bt) * S
        D = -q
        if float(np.sum(G * D)) >= 0.0:
            D = -G
            hist = []
        q1, q2, q3, q4 = quartic_coefficients(prob, U, D, z, lam, rho)
        alpha = quartic_step(q1, q2, q3, q4)
        if alpha <= 0.0:
            if hist:
                hist = []
                D = -G
                q1, q2, q3, q4 = quartic_coefficients(prob, U, D, z, lam, rho)
                alpha = quartic_step(q1, q2, q3, q4)
            if alpha <= 0.0:
                return U, z, it, False
        S = alpha * D
        U = U + S
        z = operators.forward(prob, U, U)
        G_new = gradient(prob, U, z, lam, rho)
        Y = G_new - G
        sy = float(np.sum(S * Y))
        if sy > 0.0:
            hist.append((S, Y, 1.0 / sy))
            if len(hist) > mem:
                hist.pop(0)
        G = G_new
        it += 1


def alm(prob, U0, lam0, opts, rho0=None, progress=None):
    """progress (optional): called with a status line after every inner solve."""
    U = np.array(U0, dtype=np.float64)
    lam = np.array(lam0, dtype=np.float64)
    nrm = operators.norms(prob)
    rho = float(rho0) if rho0 else (opts.rho0 if opts.rho0 > 0 else 1.0 / max(1.0, nrm["b_inf"]))
    r_cap = opts.rank_cap(prob.n, prob.m)
    z = operators.forward(prob, U, U)
    v = float(np.linalg.norm(z - prob.b)) / (1.0 + nrm["b_inf"])
    v_ref = math.inf
    outer = inner_total = growths = 0
    while v > opts.switch_tol and outer < opts.alm_outer_max:
        r = U.shape[1]
        cap = opts.rank_grow_iters if r < r_cap else opts.alm_inner_max
        tol = max(opts.alm_inner_rel * v, opts.alm_inner_floor)
        U, z, it, conv = lbfgs_inner(prob, U, lam, rho, tol, cap, opts.lbfgs_mem, nrm["c_fro"])
        inner_total += it
        v = float(np.linalg.norm(z - prob.b)) / (1.0 + nrm["b_inf"])
        if progress is not None:
            progress(f"ALM outer {outer}: {it} inner iterations, rank {U.shape[1]}, infeasibility {v:.3e}")
        # a hard inner solve raises the rank only while Phase I goes on: once
        # the infeasibility meets the switching tolerance the phase ends
        if not conv and r < r_cap and it >= cap and v > opts.switch_tol:
            r_new = min(int(math.ceil(opts.rank_factor * r)), r_cap)
            U = grow_rank(U, r_new, growths, opts.seed)
            growths += 1
            z = operators.forward(prob, U, U)
            v = float(np.linalg.norm(z - prob.b)) / (1.0 + nrm["b_inf"])
            continue
        if v <= opts.alm_eta * v_ref:
            lam = lam + rho * (z - prob.b)
            v_ref = v
        else:
            rho *= opts.alm_rho_factor
        outer += 1
    return dict(U=U, lam=lam, rho=rho, outer=outer, inner=inner_total, growths=growths,
                rank=U.shape[1], pinf=v)
