"""Dense primal-dual interior-point SDP solver, used only as an independent pin.

Textbook infeasible path-following method with the HKM search direction and a
Mehrotra-style predictor-corrector (Helmberg-Rendl-Vanderbei-Wolkowicz 1996;
Kojima-Shindoh-Hara 1997; Monteiro 1997), for

    min <C, X>  s.t.  <A_i, X> = b_i,  X PSD        (primal)
    max b^T y   s.t.  C - sum_i y_i A_i = S PSD      (dual)

Dense n x n matrices; meant for n up to a few hundred.  It shares no code with
the LoRADS oracle or the GPU library.
"""
from __future__ import annotations

import numpy as np


def _max_step(X, dX):
    L = np.linalg.cholesky(X)
    Li = np.linalg.inv(L)
    w = np.linalg.eigvalsh(Li @ dX @ Li.T)
    lo = w[0]
    return 1.0 if lo >= 0 else min(1.0, -1.0 / lo)


def solve(C, A, b, tol=1e-9, maxit=100, verbose=False):
    """C: (n, n); A: (m, n, n) symmetric; b: (m,).  Returns dict(X, y, S, obj)."""
    n = C.shape[0]
    m = b.size
    Af = A.reshape(m, n * n)
    X = np.eye(n)
    S = np.eye(n) * max(1.0, np.abs(C).max())
    y = np.zeros(m)
    for it in range(maxit):
        Rp = b - Af @ X.ravel()
        Rd = C - S - np.tensordot(y, A, axes=1)
        mu = np.trace(X @ S) / n
        pobj = float(np.sum(C * X)); dobj = float(b @ y)
        relgap = abs(pobj - dobj) / (1 + abs(pobj) + abs(dobj))
        pinf = np.linalg.norm(Rp) / (1 + np.linalg.norm(b))
        dinf = np.linalg.norm(Rd) / (1 + np.linalg.norm(C))
        if verbose:
            print(it, pobj, dobj, relgap, pinf, dinf)
        if max(relgap, pinf, dinf) < tol:
            break
        Si = np.linalg.inv(S)
        Si = (Si + Si.T) / 2
        # Schur complement M_ij = tr(A_i X A_j S^-1)
        XA = np.einsum("ab,jbc->jac", X, A)           # X A_j
        XASi = np.einsum("jac,cd->jad", XA, Si)       # X A_j S^-1
        M = np.einsum("iad,jda->ij", A, XASi)
        M = (M + M.T) / 2

        def direction(Rc):
            G = X @ Rd @ Si
            G = (G + G.T) / 2
            H = Rc @ Si
            H = (H + H.T) / 2
            # derivation: A(dX) = Rp, dS = Rd - A*(dy), dX = (Rc - X dS) S^-1 (symmetrised)
            # => A((Rc - X (Rd - A*dy)) S^-1) = Rp => M dy = Rp - A(Rc S^-1) + A(X Rd S^-1)
            rhs = Rp - Af @ H.ravel() + Af @ G.ravel()
            dy = np.linalg.solve(M, rhs)
            dS = Rd - np.tensordot(dy, A, axes=1)
            dX = (Rc - X @ dS) @ Si
            dX = (dX + dX.T) / 2
            return dX, dy, dS

        # predictor
        dX, dy, dS = direction(-X @ S)
        try:
            ap = _max_step(X, dX); ad = _max_step(S, dS)
        except np.linalg.LinAlgError:   # iterate at the rounding floor
            break
        mu_aff = np.trace((X + ap * dX) @ (S + ad * dS)) / n
        sigma = min(1.0, (mu_aff / mu) ** 3)
        # corrector
        Rc = sigma * mu * np.eye(n) - X @ S - dX @ dS
        dX, dy, dS = direction(Rc)
        try:
            ap = min(1.0, 0.98 * _max_step(X, dX)); ad = min(1.0, 0.98 * _max_step(S, dS))
        except np.linalg.LinAlgError:
            break
        X = X + ap * dX; X = (X + X.T) / 2
        y = y + ad * dy
        S = S + ad * dS; S = (S + S.T) / 2
    return dict(X=X, y=y, S=S, obj=float(np.sum(C * X)), dobj=float(b @ y), iters=it)
