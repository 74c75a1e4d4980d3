"""Reverse-mode derivatives of inverse factorization for a linear loss
L = tr(G^T Z).  Test infrastructure only.

Convention: the returned S-bar is symmetric, sym(dL/dS) = (A + A^T) / 2, so
that dL = <S-bar, E> for every symmetric perturbation E of S.

The iteration's derivative is taken through the regular (non-localized)
recurrence of eq. refinement_nonlocal, which produces the same iterates as the
localized one in exact arithmetic; no truncation (tau = 0).  The iteration
counts are inputs (frozen), since the stopping rule is not differentiable.
"""
from __future__ import annotations

import numpy as np

from .closed_forms import inv_sqrt
from .refinement import coefficients, split_point, inverse_cholesky


def sym(A: np.ndarray) -> np.ndarray:
    return 0.5 * (A + A.T)


def refine_forward(S, Z0, m, iterations):
    """Regular refinement for a fixed number of steps; returns the list
    [Z_0, ..., Z_K] (the per-iteration checkpoints)."""
    bk = coefficients(m)
    I = np.eye(S.shape[0])
    Zs = [Z0]
    Z = Z0
    for _ in range(iterations):
        delta = I - Z.T @ S @ Z
        P = bk[m] * I
        for j in range(m - 1, -1, -1):
            P = bk[j] * I + delta @ P
        Z = Z @ P
        Zs.append(Z)
    return Zs


def refine_backward(S, Zs, m, Zbar):
    """Reverse sweep of ``refine_forward``.  Given dL/dZ_K, returns
    (dL/dZ_0, A) with A the unsymmetrized dL/dS of the sweep.

    Per step, Z' = Z P with P = H_0, H_k = b_k I + delta H_{k+1}, H_m = b_m I,
    delta = I - Z^T S Z:
        Zbar_prev = Zbar P^T,  Pbar = Z^T Zbar,
        Horner reverse: deltabar += Hbar_k H_{k+1}^T, Hbar_{k+1} = delta^T Hbar_k,
        Zbar_prev -= S Z (deltabar + deltabar^T),  Sbar -= Z deltabar Z^T.
    """
    bk = coefficients(m)
    I = np.eye(S.shape[0])
    Sbar = np.zeros_like(S)
    for i in range(len(Zs) - 2, -1, -1):
        Z = Zs[i]
        delta = I - Z.T @ S @ Z
        H = [None] * (m + 1)
        H[m] = bk[m] * I
        for j in range(m - 1, -1, -1):
            H[j] = bk[j] * I + delta @ H[j + 1]
        P = H[0]
        Zbar_prev = Zbar @ P.T
        Hbar = Z.T @ Zbar
        dbar = np.zeros_like(S)
        for j in range(0, m):
            dbar += Hbar @ H[j + 1].T
            Hbar = delta.T @ Hbar
        Zbar_prev -= S @ Z @ (dbar + dbar.T)
        Sbar -= Z @ dbar @ Z.T
        Zbar = Zbar_prev
    return Zbar, Sbar


def irsi_grad(S, G, c, m, iterations):
    """sym(dL/dS) of IRSI with a fixed scale c (Z_0 = c I held constant)."""
    Zs = refine_forward(S, c * np.eye(S.shape[0]), m, iterations)
    _, A = refine_backward(S, Zs, m, G)
    return sym(A)


def inverse_cholesky_grad(S, Zbar):
    """sym(dL/dS) of the inverse Cholesky factor Z = U^{-1}, S = U^T U.

    From Z^T dS Z = X + X^T with X = dU Z upper triangular:
    dZ = -Z Phi(Z^T dS Z), Phi = upper triangle with halved diagonal, hence
    dL/dS = -Z Phi(Z^T Zbar) Z^T.
    """
    Z = inverse_cholesky(S)
    W = Z.T @ Zbar
    Phi = np.triu(W, 1) + 0.5 * np.diag(np.diag(W))
    return sym(-Z @ Phi @ Z.T)


def lif_forward_regular(S, b, base_rows, m, iters):
    """Localized-inverse-factorization tree with the regular recurrence and
    frozen per-node iteration counts.  ``iters`` maps (lo, hi) -> K.  Returns
    (Z, cache) with cache[(lo, hi)] = (Z_0 checkpoints list or leaf Z)."""
    cache = {}

    def rec(lo, hi):
        Sn = S[lo:hi, lo:hi]
        rows = hi - lo
        if rows <= base_rows:
            Z = inverse_cholesky(Sn)
            cache[(lo, hi)] = Z
            return Z
        h = split_point(rows, b)
        ZA = rec(lo, lo + h)
        ZC = rec(lo + h, hi)
        Z0 = np.zeros((rows, rows))
        Z0[:h, :h] = ZA
        Z0[h:, h:] = ZC
        Zs = refine_forward(Sn, Z0, m, iters[(lo, hi)])
        cache[(lo, hi)] = Zs
        return Zs[-1]

    Z = rec(0, S.shape[0])
    return Z, cache


def lif_grad(S, G, b, base_rows, m, iters):
    """sym(dL/dS) of localized inverse factorization through the regular
    recurrence with frozen iteration counts (``iters`` as in
    ``lif_forward_regular``).  The refinement at a node passes the diagonal
    blocks of dL/dZ_0 to its children; the leaves use
    ``inverse_cholesky_grad``."""
    _, cache = lif_forward_regular(S, b, base_rows, m, iters)
    Sbar = np.zeros_like(S)

    def rec(lo, hi, Zbar):
        Sn = S[lo:hi, lo:hi]
        rows = hi - lo
        if rows <= base_rows:
            Sbar[lo:hi, lo:hi] += inverse_cholesky_grad(Sn, Zbar)
            return
        h = split_point(rows, b)
        Z0bar, A = refine_backward(Sn, cache[(lo, hi)], m, Zbar)
        Sbar[lo:hi, lo:hi] += sym(A)
        rec(lo, lo + h, Z0bar[:h, :h])
        rec(lo + h, hi, Z0bar[h:, h:])

    rec(0, S.shape[0], G)
    return Sbar


# ----------------------------------------------------------------------------
# references through eigendecomposition (the exact limits)
# ----------------------------------------------------------------------------

def _inv_sqrt_divided_differences(lam):
    r = np.sqrt(lam)
    return -1.0 / (r[:, None] * r[None, :] * (r[:, None] + r[None, :]))


def inv_sqrt_grad(S, G):
    """sym(dL/dS) for Z = S^{-1/2} (the IRSI limit): with S = Q diag(lam) Q^T,
    dZ = Q (F o (Q^T dS Q)) Q^T and F_ij the divided differences of
    lam^{-1/2}, so dL/dS = Q (F o (Q^T G Q)) Q^T."""
    lam, Q = np.linalg.eigh(S)
    F = _inv_sqrt_divided_differences(lam)
    return sym(Q @ (F * (Q.T @ sym(G) @ Q)) @ Q.T)


def lif_limit_grad(S, G, b, base_rows):
    """sym(dL/dS) of the exact LIF limit Z = Z_0 W^{-1/2}, W = Z_0^T S Z_0,
    by the chain rule with the eigendecomposition derivative of W^{-1/2}."""
    Sbar = np.zeros_like(S)

    def fwd(lo, hi):
        Sn = S[lo:hi, lo:hi]
        rows = hi - lo
        if rows <= base_rows:
            return inverse_cholesky(Sn)
        h = split_point(rows, b)
        Z0 = np.zeros((rows, rows))
        Z0[:h, :h] = fwd(lo, lo + h)
        Z0[h:, h:] = fwd(lo + h, hi)
        return Z0 @ inv_sqrt(Z0.T @ Sn @ Z0)

    def rec(lo, hi, Zbar):
        Sn = S[lo:hi, lo:hi]
        rows = hi - lo
        if rows <= base_rows:
            Sbar[lo:hi, lo:hi] += inverse_cholesky_grad(Sn, Zbar)
            return
        h = split_point(rows, b)
        Z0 = np.zeros((rows, rows))
        Z0[:h, :h] = fwd(lo, lo + h)
        Z0[h:, h:] = fwd(lo + h, hi)
        W = Z0.T @ Sn @ Z0
        lam, Q = np.linalg.eigh(W)
        Wm = (Q * lam ** -0.5) @ Q.T
        Z0bar = Zbar @ Wm
        F = _inv_sqrt_divided_differences(lam)
        V = Z0.T @ Zbar
        Wbar = Q @ (F * (Q.T @ V @ Q)) @ Q.T
        Z0bar += Sn @ Z0 @ (Wbar + Wbar.T)
        Sbar[lo:hi, lo:hi] += sym(Z0 @ Wbar @ Z0.T)
        rec(lo, lo + h, Z0bar[:h, :h])
        rec(lo + h, hi, Z0bar[h:, h:])

    rec(0, S.shape[0], G)
    return Sbar
