"""Dense FP64 oracle of iterative refinement, localized inverse factorization
and recursive inverse Cholesky, with the paper's leaf-block truncation.

Test infrastructure only (see the package docstring).

Conventions
-----------
* Matrices are real symmetric; the conjugate transpose of the paper is the
  plain transpose here.
* Block grid: b x b blocks from the matrix origin; a sub-problem always starts
  on a block boundary, so its blocks are blocks of the global grid.  The last
  block row/column may be partial.
* Truncation (Sec. 5): after every matrix-matrix product and after every leaf
  (base) factorization, blocks whose Frobenius norm is below tau are set to
  zero; a block whose norm equals tau is kept.  S itself is truncated the same
  way before it is factorized.  Sums, differences and scalings are not
  truncated.  tau = 0 truncates nothing.
* m: the refinement order (the paper uses m = 4).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


class NoConvergence(RuntimeError):
    pass


class NotPositiveDefinite(RuntimeError):
    pass


# ----------------------------------------------------------------------------
# basic pieces
# ----------------------------------------------------------------------------

def coefficients(m: int) -> list[float]:
    """b_0 = 1, b_k = (2k - 1) / (2k) * b_{k-1} (eq. refinement_nonlocal)."""
    b = [1.0]
    for k in range(1, m + 1):
        b.append((2 * k - 1) / (2 * k) * b[-1])
    return b


def block_norms(X: np.ndarray, b: int) -> np.ndarray:
    """Frobenius norm of every b x b block of X (partial edge blocks included)."""
    r, c = X.shape
    nbr, nbc = (r + b - 1) // b, (c + b - 1) // b
    P = np.zeros((nbr * b, nbc * b))
    P[:r, :c] = X
    T = P.reshape(nbr, b, nbc, b)
    return np.sqrt(np.einsum("ikjl,ikjl->ij", T, T))


def truncate(X: np.ndarray, b: int, tau: float) -> np.ndarray:
    """Zero every b x b block of X whose Frobenius norm is < tau (Sec. 5)."""
    if tau <= 0.0:
        return X
    keep = block_norms(X, b) >= tau
    mask = np.repeat(np.repeat(keep, b, axis=0), b, axis=1)[: X.shape[0], : X.shape[1]]
    return np.where(mask, X, 0.0)


def round_to(X: np.ndarray, prec: str) -> np.ndarray:
    """Input rounding of the precision form (values returned as FP64).

    ``"fp32"``: round to nearest even FP32.  ``"bf16"``: round to FP32 first,
    then to BF16 by round to nearest even on the 32-bit pattern (add 0x7FFF
    plus the lowest kept bit, drop the low 16 bits); infinities and NaN keep
    their high half.  ``"fp64"``: unchanged.
    """
    if prec == "fp64":
        return X
    f = np.asarray(X, dtype=np.float64).astype(np.float32)
    if prec == "fp32":
        return f.astype(np.float64)
    if prec != "bf16":
        raise ValueError(prec)
    u = f.view(np.uint32).astype(np.uint64)
    special = (u & 0x7F800000) == 0x7F800000
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    kept = np.where(special, (u >> 16) << 16, rounded) & 0xFFFFFFFF
    return kept.astype(np.uint32).view(np.float32).astype(np.float64)


def mult(A: np.ndarray, B: np.ndarray, b: int, tau: float, prec: str = "fp64") -> np.ndarray:
    """A matrix-matrix product followed by truncation.  With ``prec`` fp32 or
    bf16 the inputs are rounded first (the precision form: reduced-precision
    inputs, the products of the rounded values summed, FP64 result)."""
    return truncate(round_to(A, prec) @ round_to(B, prec), b, tau)


def mult_add(A: np.ndarray, B: np.ndarray, b: int, tau: float, prec: str = "fp64", alpha: float = 1.0,
             D: np.ndarray | None = None, gamma: float = 0.0) -> np.ndarray:
    """trunc(alpha A B + gamma D): a product with an added term, truncated as a
    whole.  This is how a Horner step delta T with T = X + c I is read in the
    precision form: only the stored part X (and delta) enter the product in
    the input precision; the identity part contributes c delta, added in FP64
    (the identity itself is exact in any precision, so rounding it together
    with X would add an error that the product does not need).  ``alpha``
    scales the product of the rounded inputs (the first Horner step
    b_m delta delta).  In FP64 this is trunc(A (alpha B) + gamma D), equal to
    ``mult`` of the explicit factor up to the order of the sums."""
    P = round_to(A, prec) @ round_to(B, prec)
    if alpha != 1.0:
        P = alpha * P
    if D is not None and gamma != 0.0:
        P = P + gamma * D
    return truncate(P, b, tau)


def gershgorin_bound(S: np.ndarray) -> float:
    """Gershgorin upper bound of the spectral radius: max_i sum_j |S_ij|
    (Sec. 2.2, scaling of the identity start)."""
    return float(np.max(np.sum(np.abs(S), axis=1)))


def start_scale(S: np.ndarray, mode: str, value: float | None = None) -> float:
    """Scale c of the start Z_0 = c I (Sec. 2.2).

    * ``"sqrt2_over_gersh"``: c = sqrt(2 / beta), beta the Gershgorin bound
      (the paper's choice);
    * ``"inv_sqrt_gersh"``: c = 1 / sqrt(beta);
    * ``"inv_sqrt_lmax"``: c = 1 / sqrt(value), value = lambda_max;
    * ``"optimal"``: c = sqrt(2 / (lambda_min + lambda_max)) from eigvalsh;
    * ``"given"``: c = value.
    """
    if mode == "sqrt2_over_gersh":
        return math.sqrt(2.0 / gershgorin_bound(S))
    if mode == "inv_sqrt_gersh":
        return 1.0 / math.sqrt(gershgorin_bound(S))
    if mode == "inv_sqrt_lmax":
        return 1.0 / math.sqrt(value)
    if mode == "optimal":
        ev = np.linalg.eigvalsh(S)
        return math.sqrt(2.0 / (ev[0] + ev[-1]))
    if mode == "given":
        return float(value)
    raise ValueError(mode)


def inverse_cholesky(S: np.ndarray) -> np.ndarray:
    """Upper-triangular Z with Z^T S Z = I: S = U^T U (Cholesky), Z = U^{-1}.
    This is the leaf factorization S^{-1} = Z Z^T of Alg. 1 and Alg. 2."""
    try:
        L = np.linalg.cholesky(S)
    except np.linalg.LinAlgError as e:
        raise NotPositiveDefinite(str(e)) from e
    U = L.T
    n = S.shape[0]
    return np.linalg.solve(U, np.eye(n)) if n else np.zeros((0, 0))


def split_point(rows: int, b: int) -> int:
    """Rows of the leading part A when a range of ``rows`` rows is split: the
    range's ceil(nb/2) leading blocks, nb = ceil(rows / b)."""
    nb = (rows + b - 1) // b
    return ((nb + 1) // 2) * b


# ----------------------------------------------------------------------------
# refinement
# ----------------------------------------------------------------------------

@dataclass
class RefineInfo:
    iterations: int = 0
    norms: list = field(default_factory=list)     # ||delta_k||_F, k = 1..iterations
    stagnated: bool = False
    reduced: list = field(default_factory=list)   # per iteration: correction in reduced precision


def check_divergence(k: int, e: float, e_prev: float | None) -> None:
    """A non-finite norm, or one that grows while >= 1, means divergence."""
    if not math.isfinite(e):
        raise NoConvergence(f"non-finite ||delta|| at iteration {k}")
    if e_prev is not None and e > e_prev and e >= 1.0:
        raise NoConvergence(f"||delta|| grew from {e_prev:g} to {e:g} at iteration {k}")


def stop_now(k: int, e: float, e_prev: float | None, m: int, stop: str, tol: float) -> bool:
    """Stop decision after delta_k has been formed (k >= 1).

    ``"paper"``: stop when ||delta_k||_F > ||delta_{k-1}||_F^{m+1}, first tested
    at k = 2 (the error record starts at the largest real value and its
    (m+1)-th power), or when delta_k = 0.  ``"tol"``: stop when
    ||delta_k||_F <= tol, or when the norm stops decreasing.  A norm that grows
    while >= 1 means divergence.
    """
    check_divergence(k, e, e_prev)
    if stop == "paper":
        if e == 0.0:
            return True
        return e_prev is not None and e > e_prev ** (m + 1)
    if stop == "tol":
        if e <= tol:
            return True
        return e_prev is not None and e >= e_prev
    raise ValueError(stop)


def upper_blocks(A: np.ndarray, b: int, strict: bool = False) -> np.ndarray:
    """A with every b x b block below the block diagonal zeroed (and the
    diagonal blocks too when ``strict``)."""
    n = A.shape[0]
    I, J = np.meshgrid(np.arange(n) // b, np.arange(n) // b, indexing="ij")
    keep = J > I if strict else J >= I
    return np.where(keep, A, 0.0)


def localized_refinement(S, Z0, delta0, b, tau, m=4, stop="paper", tol=0.0, max_iter=100, info=None,
                         prec="fp64", prec_switch=0.0, sym_delta=False, update_prec="fp64", trace=None):
    """Localized iterative refinement (eq. refinement_local; Alg. 2 repeat loop).

    Each iteration, with T_k the Horner terms of sum_{k=1}^m b_k delta^k:
        T = b_{m-1} I + b_m delta
        T = b_k I + delta T          (k = m-2, ..., 1; product truncated)
        q = delta T                  (truncated)
        M = Z q                      (truncated)
        Z' = Z + M
        SM = S M                     (truncated)
        delta' = delta - Z'^T SM - SM^T Z      (each product truncated;
                                                M^T S is formed as (SM)^T)
    ``prec`` applies to the products that form M (delta T and Z q); the
    delta-update products stay FP64, so delta keeps tracking I - Z^T S Z.
    In reduced precision a Horner factor T = X + c I is not rounded as a
    whole: delta T = delta X + c delta with delta and X rounded and the
    identity part c delta added in FP64 (``mult_add``).
    ``prec_switch`` > 0 is the precision schedule: an iteration uses ``prec``
    only while ||delta||_F before it exceeds ``prec_switch`` and FP64 after;
    an inexact correction converges linearly, so the stopping rule is applied
    to the FP64 iterations only (reduced ones are checked for divergence).
    With ``prec_switch`` = 0 every iteration uses ``prec`` and is tested.
    ``sym_delta``: delta is symmetric in exact arithmetic, so only its upper
    block triangle is updated (the blocks (I, J), J >= I, of the two
    truncated products) and the strictly upper part is mirrored below.
    ``update_prec`` (with ``prec_switch`` > 0): the delta-update products of
    the reduced iterations (S M, Z'^T SM, SM^T Z) in that input precision
    too.  delta then no longer tracks I - Z^T S Z to FP64 accuracy, so when
    the schedule moves to FP64 it is formed again from its definition,
    delta = I - trunc(Z^T trunc(S Z)) in FP64 (S Z first, as the update
    forms S M; mirrored like an update with ``sym_delta``); its norm
    replaces the last recorded one, which the stopping rule then compares
    against.
    ``trace`` (tests): called as trace(k, event, Z, delta) with event
    "recomputed" (delta formed again before iteration k) or "updated" (Z and
    delta after iteration k).
    Returns (Z, RefineInfo).
    """
    info = info if info is not None else RefineInfo()
    bk = coefficients(m)
    n = S.shape[0]
    I = np.eye(n)
    Z, delta = Z0.copy(), delta0.copy()
    if not np.any(delta):
        return Z, info
    assert update_prec == "fp64" or prec_switch > 0.0, "a reduced delta update needs the precision schedule"
    e_prev = None
    e_cur = float(np.sqrt(np.sum(delta * delta)))
    stale = False  # delta carries the rounding of reduced-precision updates
    for k in range(1, max_iter + 1):
        reduced = prec != "fp64" and (prec_switch == 0.0 or e_cur > prec_switch)
        p = prec if reduced else "fp64"
        if stale and not reduced:
            delta = I - mult(Z.T, mult(S, Z, b, tau), b, tau)
            if sym_delta:
                U = upper_blocks(delta, b)
                delta = U + upper_blocks(U, b, strict=True).T
            e_cur = float(np.sqrt(np.sum(delta * delta)))
            info.norms[-1] = e_cur
            e_prev = e_cur
            stale = False
            if trace:
                trace(k, "recomputed", Z, delta)
        if m == 1:
            q = bk[1] * delta
        elif p == "fp64":
            T = bk[m - 1] * I + bk[m] * delta
            for j in range(m - 2, 0, -1):
                T = bk[j] * I + mult(delta, T, b, tau, p)
            q = mult(delta, T, b, tau, p)
        else:
            # reduced precision: T_j = X_j + b_j I with only X_j (and delta)
            # rounded; delta T_j = delta X_j + b_j delta, the second term FP64
            X = mult_add(delta, delta, b, tau, p, alpha=bk[m], D=delta, gamma=bk[m - 1])
            for j in range(m - 2, 0, -1):
                X = mult_add(delta, X, b, tau, p, D=delta, gamma=bk[j])
            q = X
        M = mult(Z, q, b, tau, p)
        Z_new = Z + M
        pu = update_prec if reduced else "fp64"
        SM = mult(S, M, b, tau, pu)
        X1 = mult(Z_new.T, SM, b, tau, pu)
        X2 = mult(SM.T, Z, b, tau, pu)
        stale = pu != "fp64"
        delta = delta - X1 - X2
        if sym_delta:
            U = upper_blocks(delta, b)
            delta = U + upper_blocks(U, b, strict=True).T
        Z = Z_new
        if trace:
            trace(k, "updated", Z, delta)
        e = float(np.sqrt(np.sum(delta * delta)))
        info.norms.append(e)
        info.reduced.append(reduced)
        info.iterations = k
        if prec_switch > 0.0 and reduced:
            check_divergence(k, e, e_prev)
        elif stop_now(k, e, e_prev, m, stop, tol):
            if stop == "tol" and e > tol:
                info.stagnated = True
            return Z, info
        e_prev = e
        e_cur = e
    raise NoConvergence(f"no convergence in {max_iter} iterations")


def nonlocal_refinement(S, Z0, b, tau, m=4, iterations=None, stop="paper", tol=0.0, max_iter=100):
    """Regular (non-localized) refinement, eq. refinement_nonlocal:
    delta_i = I - (Z_i^T S) Z_i, Z_{i+1} = Z_i P_i with
    P_i = sum_{k=0}^m b_k delta_i^k in Horner form (every product truncated).
    With ``iterations`` given, exactly that many steps are taken.
    Returns (Z, RefineInfo)."""
    bk = coefficients(m)
    n = S.shape[0]
    I = np.eye(n)
    info = RefineInfo()
    Z = Z0.copy()
    delta = I - mult(mult(Z.T, S, b, tau), Z, b, tau)
    if iterations is None and not np.any(delta):
        return Z, info
    e_prev = None
    for k in range(1, (iterations if iterations is not None else max_iter) + 1):
        P = bk[m] * I
        for j in range(m - 1, -1, -1):
            P = bk[j] * I + mult(delta, P, b, tau)
        Z = mult(Z, P, b, tau)
        delta = I - mult(mult(Z.T, S, b, tau), Z, b, tau)
        e = float(np.sqrt(np.sum(delta * delta)))
        info.norms.append(e)
        info.iterations = k
        if iterations is None and stop_now(k, e, e_prev, m, stop, tol):
            return Z, info
        e_prev = e
    if iterations is None:
        raise NoConvergence(f"no convergence in {max_iter} iterations")
    return Z, info


# ----------------------------------------------------------------------------
# the three methods
# ----------------------------------------------------------------------------

def irsi(S, b, tau, m=4, start="sqrt2_over_gersh", start_value=None, stop="paper", tol=0.0,
         max_iter=100, truncate_input=True, prec="fp64", refinement="local", prec_switch=0.0,
         sym_delta=False, update_prec="fp64"):
    """Iterative refinement from a scaled identity (IRSI, Sec. 2.2):
    Z_0 = c I, delta_0 = I - c^2 S (a scaling, no product), then localized
    refinement.  With ``refinement="nonlocal"`` the regular form of
    eq. refinement_nonlocal runs from the same Z_0 instead (its delta_0 is
    then I - (Z_0^T S) Z_0 with both products truncated).
    Returns (Z, RefineInfo, c)."""
    St = truncate(S, b, tau) if truncate_input else S
    c = start_scale(St, start, start_value)
    n = S.shape[0]
    Z0 = c * np.eye(n)
    if refinement == "nonlocal":
        assert prec == "fp64", "the regular form is FP64 only"
        Z, info = nonlocal_refinement(St, Z0, b, tau, m, stop=stop, tol=tol, max_iter=max_iter)
        return Z, info, c
    assert refinement == "local", refinement
    delta0 = np.eye(n) - (c * c) * St
    Z, info = localized_refinement(St, Z0, delta0, b, tau, m, stop, tol, max_iter, prec=prec,
                                   prec_switch=prec_switch, sym_delta=sym_delta, update_prec=update_prec)
    return Z, info, c


@dataclass
class LifNode:
    lo: int                      # first row (multiple of b)
    hi: int                      # one past the last row
    depth: int
    children: tuple = ()
    info: RefineInfo | None = None
    delta0_norm2: float = 0.0    # ||delta_0||_2 of this node's refinement


def lif_plan(n: int, b: int, base_rows: int) -> LifNode:
    """Binary split tree: a range is split at ceil(nb/2) blocks while it has
    more than ``base_rows`` rows."""
    def build(lo, hi, depth):
        node = LifNode(lo, hi, depth)
        if hi - lo > base_rows:
            h = lo + split_point(hi - lo, b)
            node.children = (build(lo, h, depth + 1), build(h, hi, depth + 1))
        return node
    return build(0, n, 0)


def lif(S, b, tau, m=4, base_rows=4096, stop="paper", tol=0.0, max_iter=100, truncate_input=True,
        plan=None, prec="fp64", refinement="local", prec_switch=0.0, sym_delta=False, update_prec="fp64"):
    """Localized inverse factorization (Alg. 2) with an inverse Cholesky leaf.

    For a node with children A (leading rows) and C:
        Z_A = lif(A), Z_C = lif(C), Z_0 = diag(Z_A, Z_C),
        X = (Z_A^T B) Z_C (each product truncated),
        delta_0 = -[[0, X], [X^T, 0]],
        then localized refinement of Z_0 on the node's S.
    With ``refinement="nonlocal"`` (recursive inverse factorization with the
    regular correction, Sec. 2.3): each node is corrected by the regular form
    of eq. refinement_nonlocal from the same Z_0, whose delta_0 is
    I - (Z_0^T S) Z_0 (products truncated); X is not formed.
    Returns (Z, plan) with per-node RefineInfo stored in the plan.
    """
    assert refinement in ("local", "nonlocal"), refinement
    assert refinement == "local" or prec == "fp64", "the regular form is FP64 only"
    St = truncate(S, b, tau) if truncate_input else S
    plan = plan if plan is not None else lif_plan(S.shape[0], b, base_rows)

    def rec(node):
        Sn = St[node.lo:node.hi, node.lo:node.hi]
        if not node.children:
            return truncate(inverse_cholesky(Sn), b, tau)
        a, c = node.children
        ZA = rec(a)
        ZC = rec(c)
        h = a.hi - a.lo
        rows = node.hi - node.lo
        Z0 = np.zeros((rows, rows))
        Z0[:h, :h] = ZA
        Z0[h:, h:] = ZC
        if refinement == "nonlocal":
            node.info = RefineInfo()
            Z, node.info = nonlocal_refinement(Sn, Z0, b, tau, m, stop=stop, tol=tol, max_iter=max_iter)
            return Z
        B = Sn[:h, h:]
        X = mult(mult(ZA.T, B, b, tau), ZC, b, tau)
        delta0 = np.zeros((rows, rows))
        delta0[:h, h:] = -X
        delta0[h:, :h] = -X.T
        node.delta0_norm2 = float(np.linalg.norm(delta0, 2)) if rows <= 4000 else float("nan")
        node.info = RefineInfo()
        Z, _ = localized_refinement(Sn, Z0, delta0, b, tau, m, stop, tol, max_iter, node.info, prec=prec,
                                    prec_switch=prec_switch, sym_delta=sym_delta, update_prec=update_prec)
        return Z

    return rec(plan), plan


def rinch(S, b, tau, base_rows=4096, truncate_input=True):
    """Recursive inverse Cholesky (Alg. 1), split as in ``lif_plan``:
        Z00 = rinch(S00); R = Z00^T S01; Q = S11 - R^T R; Z11 = rinch(Q);
        Z01 = -(Z00 R) Z11; Z10 = 0.
    Every product is truncated, and so is every leaf result."""
    St = truncate(S, b, tau) if truncate_input else S

    def rec(Sn):
        rows = Sn.shape[0]
        if rows <= base_rows:
            return truncate(inverse_cholesky(Sn), b, tau)
        h = split_point(rows, b)
        S00, S01, S11 = Sn[:h, :h], Sn[:h, h:], Sn[h:, h:]
        Z00 = rec(S00)
        R = mult(Z00.T, S01, b, tau)
        Q = S11 - mult(R.T, R, b, tau)
        Z11 = rec(Q)
        Z01 = -mult(mult(Z00, R, b, tau), Z11, b, tau)
        Z = np.zeros((rows, rows))
        Z[:h, :h] = Z00
        Z[:h, h:] = Z01
        Z[h:, h:] = Z11
        return Z

    return rec(St)


def true_residual(S, Z) -> float:
    """||I - Z^T S Z||_F, untruncated (Table 1's error measure)."""
    R = np.eye(S.shape[0]) - Z.T @ S @ Z
    return float(np.sqrt(np.sum(R * R)))
