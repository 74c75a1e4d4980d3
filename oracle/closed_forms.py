"""Exact results the refinement-based methods reach, and quantities that
predict their iterates.  Test infrastructure only.

None of these functions runs the refinement iteration: they are the plain
mathematical definitions the iteration is pinned against.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def binomial_coefficients(m: int) -> list[Fraction]:
    """Taylor coefficients of (1 - x)^{-1/2}: C(2k, k) / 4^k, k = 0..m.
    The refinement multiplies Z by a truncated series of this function
    (eq. refinement_nonlocal)."""
    return [Fraction(math.comb(2 * k, k), 4 ** k) for k in range(m + 1)]


def inv_sqrt(S: np.ndarray) -> np.ndarray:
    """Loewdin inverse square root S^{-1/2} by eigendecomposition: the limit of
    refinement from a scaled identity (Sec. 2.2)."""
    lam, Q = np.linalg.eigh(S)
    return (Q * lam ** -0.5) @ Q.T


def upper_inverse_factor_check(S: np.ndarray, Z: np.ndarray) -> tuple[float, float, float]:
    """(max |strict lower part of Z|, min diag(Z), ||Z^T S Z - I||_F): an upper
    triangular Z with positive diagonal and Z^T S Z = I is the unique inverse
    Cholesky factor."""
    low = float(np.max(np.abs(np.tril(Z, -1)))) if Z.size else 0.0
    dmin = float(np.min(np.diag(Z))) if Z.size else 1.0
    R = Z.T @ S @ Z - np.eye(S.shape[0])
    return low, dmin, float(np.sqrt(np.sum(R * R)))


def lif_limit(S: np.ndarray, b: int, base_rows: int) -> np.ndarray:
    """Untruncated limit of localized inverse factorization with an inverse
    Cholesky leaf: for a node with children A and C,
        Z_0 = diag(Z_A, Z_C),  Z = Z_0 (Z_0^T S Z_0)^{-1/2},
    the fixed point of refinement started from Z_0 (Sec. 2.3), computed by
    eigendecomposition.  The leaf factor is pinned through
    ``upper_inverse_factor_check``."""
    rows = S.shape[0]
    if rows <= base_rows:
        U = np.linalg.cholesky(S).T
        return np.linalg.inv(U)
    nb = (rows + b - 1) // b
    h = ((nb + 1) // 2) * b
    Z0 = np.zeros_like(S)
    Z0[:h, :h] = lif_limit(S[:h, :h], b, base_rows)
    Z0[h:, h:] = lif_limit(S[h:, h:], b, base_rows)
    return Z0 @ inv_sqrt(Z0.T @ S @ Z0)


def spectral_map(x, m: int):
    """One refinement step acts on each eigenvalue x of delta as
    f(x) = 1 - (1 - x) p(x)^2, p(x) = sum_{k<=m} C(2k,k)/4^k x^k."""
    c = [float(v) for v in binomial_coefficients(m)]
    p = np.zeros_like(np.asarray(x, dtype=float))
    for k in range(m, -1, -1):
        p = p * x + c[k]
    return 1.0 - (1.0 - x) * p * p


def predicted_norms(mu: np.ndarray, m: int, iterations: int) -> list[float]:
    """||delta_k||_F, k = 1..iterations, predicted from the eigenvalues ``mu``
    of delta_0 by repeated application of ``spectral_map``."""
    out = []
    x = np.asarray(mu, dtype=float)
    for _ in range(iterations):
        x = spectral_map(x, m)
        out.append(float(np.sqrt(np.sum(x * x))))
    return out


def k_max(eps: float, lam_min: float, lam_max: float, m: int) -> int:
    """Iteration bound of eq. iter_refine_no_of_iters (Sec. 3.3):
    ceil( log( log(eps) / log(1 - lam_min/lam_max) ) / log(m + 1) )."""
    return math.ceil(math.log(math.log(eps) / math.log(1.0 - lam_min / lam_max)) / math.log(m + 1))
