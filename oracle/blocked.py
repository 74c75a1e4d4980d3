"""Block-sparse CPU oracle: the algorithms of ``refinement.py`` on block lists,
for sizes the dense oracle cannot hold (the 100,000-row chain).  Test
infrastructure only (the product path never calls it).

A matrix is a dict {(i, j): b x b FP64 block} of its nonzero blocks, with n
and b (class BM); blocks of the last block row/column are zero beyond n.
Every operation is the dense oracle's operation written over nonzero blocks:
a product sums op(A)_ik op(B)_kj over k in ascending order and drops every
output block whose Frobenius norm is < tau (Sec. 4, Sec. 5); sums and scalings
are exact blockwise; the leaf factorization is the dense oracle's
``inverse_cholesky`` on the leaf's dense part.  The refinement, LIF, IRSI and
RINCH drivers take the steps of the dense oracle in the same order, so the
two agree up to the summation order inside products (pinned by tests at
sizes both can run).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

from . import refinement as R

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbsmm.so")
_lib = None


@dataclass
class BM:
    n: int
    b: int
    blocks: dict = field(default_factory=dict)

    @property
    def nb(self) -> int:
        return (self.n + self.b - 1) // self.b

    def rows(self) -> dict:
        """{i: sorted columns of block row i}."""
        out: dict = {}
        for (i, j) in self.blocks:
            out.setdefault(i, []).append(j)
        for v in out.values():
            v.sort()
        return out


def from_blocks(M) -> BM:
    A = BM(int(M.n), int(M.b))
    for r, c, v in zip(np.asarray(M.brow).tolist(), np.asarray(M.bcol).tolist(), np.asarray(M.vals)):
        A.blocks[(r, c)] = np.array(v, dtype=np.float64)
    return A


def to_arrays(A: BM):
    """(brow, bcol, vals) sorted by (row, col)."""
    keys = sorted(A.blocks)
    brow = np.array([k[0] for k in keys], np.int32)
    bcol = np.array([k[1] for k in keys], np.int32)
    vals = np.stack([A.blocks[k] for k in keys]) if keys else np.zeros((0, A.b, A.b))
    return brow, bcol, vals


def to_dense(A: BM) -> np.ndarray:
    nb, b = A.nb, A.b
    D = np.zeros((nb * b, nb * b))
    for (i, j), v in A.blocks.items():
        D[i * b:(i + 1) * b, j * b:(j + 1) * b] = v
    return D[:A.n, :A.n]


def _norm(v: np.ndarray) -> float:
    return float(np.sqrt(np.sum(v * v)))


def truncate(A: BM, tau: float) -> BM:
    """Blocks with Frobenius norm < tau removed (Sec. 5)."""
    if tau <= 0.0:
        return A
    return BM(A.n, A.b, {k: v for k, v in A.blocks.items() if _norm(v) >= tau})


def transpose(A: BM) -> BM:
    return BM(A.n, A.b, {(j, i): v.T.copy() for (i, j), v in A.blocks.items()})


def _clib():
    """The oracle's C block product (``bsmm.c``, built by ``oracle/build.py``),
    or None when it is not built."""
    global _lib
    if _lib is None and os.path.exists(_LIB_PATH):
        lib = ctypes.CDLL(_LIB_PATH)
        p = ctypes.c_void_p
        lib.bsmm_pattern.argtypes = [ctypes.c_int64, p, p, p, p, p]
        lib.bsmm_values.argtypes = [ctypes.c_int64, ctypes.c_int32, p, p, p, p, p, p, p, p, p, p]
        _lib = lib
    return _lib


def _csr(A: BM):
    """(row pointers int64, columns int32, values (nnzb, b, b)) in (row, col) order."""
    keys = sorted(A.blocks)
    nb = A.nb
    rows = np.fromiter((k[0] for k in keys), np.int64, len(keys))
    cols = np.fromiter((k[1] for k in keys), np.int32, len(keys))
    rp = np.zeros(nb + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=nb), out=rp[1:])
    vals = np.empty((len(keys), A.b, A.b))
    for e, k in enumerate(keys):
        vals[e] = A.blocks[k]
    return rp, cols, vals


def mult(A: BM, B: BM, tau: float) -> BM:
    """trunc_tau(A B): output block (i, j) = sum over k ascending of A_ik B_kj.
    Runs the oracle's C product when it is built (rows of the output on
    several threads), else the loop of ``mult_py``; the two are pinned to
    each other and to dense products by tests."""
    lib = _clib()
    if lib is None:
        return mult_py(A, B, tau)
    nb, b = A.nb, A.b
    arp, acol, avals = _csr(A)
    brp, bcol, bvals = _csr(B)
    cnt = np.zeros(nb, np.int64)
    ptr = lambda x: x.ctypes.data  # noqa: E731
    if lib.bsmm_pattern(nb, ptr(arp), ptr(acol), ptr(brp), ptr(bcol), ptr(cnt)) != 0:
        raise MemoryError("bsmm_pattern")
    crp = np.zeros(nb + 1, np.int64)
    np.cumsum(cnt, out=crp[1:])
    nc = int(crp[-1])
    ccol = np.empty(nc, np.int32)
    cvals = np.empty((nc, b, b))
    cnorm = np.empty(nc)
    if lib.bsmm_values(nb, b, ptr(arp), ptr(acol), ptr(avals), ptr(brp), ptr(bcol), ptr(bvals), ptr(crp),
                       ptr(ccol), ptr(cvals), ptr(cnorm)) != 0:
        raise MemoryError("bsmm_values")
    keep = np.ones(nc, bool) if tau <= 0.0 else cnorm >= tau
    crow = np.repeat(np.arange(nb), np.diff(crp))
    out = {}
    for e in np.nonzero(keep)[0].tolist():
        out[(int(crow[e]), int(ccol[e]))] = cvals[e]
    return BM(A.n, A.b, out)


def mult_py(A: BM, B: BM, tau: float) -> BM:
    """trunc_tau(A B): output block (i, j) = sum over k ascending of A_ik B_kj
    (plain Python loop over block products)."""
    brows = B.rows()
    out = {}
    for i, ks in sorted(A.rows().items()):
        acc: dict = {}
        for k in ks:
            a = A.blocks[(i, k)]
            for j in brows.get(k, ()):
                p = a @ B.blocks[(k, j)]
                if j in acc:
                    acc[j] += p
                else:
                    acc[j] = p
        for j, v in acc.items():
            out[(i, j)] = v
    return truncate(BM(A.n, A.b, out), tau)


def axpy(alpha: float, A: BM | None, beta: float, B: BM | None) -> BM:
    """alpha A + beta B (either may be None), exact blockwise, not truncated."""
    ref = A if A is not None else B
    out: dict = {}
    for M, s in ((A, alpha), (B, beta)):
        if M is None:
            continue
        for k, v in M.blocks.items():
            out[k] = out[k] + s * v if k in out else s * v
    return BM(ref.n, ref.b, out)


def identity(n: int, b: int, c: float, r0: int = 0, r1: int | None = None) -> BM:
    """c I on the real rows of block rows [r0, r1)."""
    nb = (n + b - 1) // b
    r1 = nb if r1 is None else r1
    out = {}
    for i in range(r0, r1):
        v = np.zeros((b, b))
        real = min(b, n - i * b)
        v[np.arange(real), np.arange(real)] = c
        out[(i, i)] = v
    return BM(n, b, out)


def restrict(A: BM, r0: int, r1: int, c0: int, c1: int) -> BM:
    """The blocks in block rows [r0, r1) and block columns [c0, c1)."""
    return BM(A.n, A.b, {(i, j): v for (i, j), v in A.blocks.items() if r0 <= i < r1 and c0 <= j < c1})


def frob(A: BM) -> float:
    return float(math.sqrt(sum(float(np.sum(v * v)) for v in A.blocks.values())))


# ----------------------------------------------------------------------------
# refinement and the three methods (same steps as refinement.py)
# ----------------------------------------------------------------------------

def localized_refinement(S: BM, Z0: BM, delta0: BM, tau: float, m: int, stop: str, tol: float, max_iter: int,
                         r0: int, r1: int):
    """eq. refinement_local on block rows [r0, r1) (the identity lives there);
    the steps of ``refinement.localized_refinement`` in FP64."""
    info = R.RefineInfo()
    bk = R.coefficients(m)
    Z, delta = Z0, delta0
    if not delta.blocks or frob(delta) == 0.0:
        return Z, info
    n, b = S.n, S.b
    e_prev = None
    for k in range(1, max_iter + 1):
        if m == 1:
            q = axpy(bk[1], delta, 0.0, None)
        else:
            T = axpy(bk[m], delta, 1.0, identity(n, b, bk[m - 1], r0, r1))
            for j in range(m - 2, 0, -1):
                T = axpy(1.0, identity(n, b, bk[j], r0, r1), 1.0, mult(delta, T, tau))
            q = mult(delta, T, tau)
        M = mult(Z, q, tau)
        Z_new = axpy(1.0, Z, 1.0, M)
        SM = mult(S, M, tau)
        X1 = mult(transpose(Z_new), SM, tau)
        X2 = mult(transpose(SM), Z, tau)
        delta = axpy(1.0, axpy(1.0, delta, -1.0, X1), -1.0, X2)
        Z = Z_new
        e = frob(delta)
        info.norms.append(e)
        info.iterations = k
        if R.stop_now(k, e, e_prev, m, stop, tol):
            if stop == "tol" and e > tol:
                info.stagnated = True
            return Z, info
        e_prev = e
    raise R.NoConvergence(f"no convergence in {max_iter} iterations")


def _leaf(St: BM, lo: int, hi: int, tau: float) -> BM:
    """Truncated upper-triangular inverse Cholesky factor of rows [lo, hi)."""
    b = St.b
    r0, r1 = lo // b, (hi + b - 1) // b
    D = np.zeros((hi - lo, hi - lo))
    for (i, j), v in St.blocks.items():
        if r0 <= i < r1 and r0 <= j < r1:
            ri, rj = i * b - lo, j * b - lo
            hr, hc = min(b, hi - i * b), min(b, hi - j * b)
            D[ri:ri + hr, rj:rj + hc] = v[:hr, :hc]
    Zd = R.inverse_cholesky(D)
    out = {}
    for i in range(r0, r1):
        for j in range(i, r1):
            v = np.zeros((b, b))
            ri, rj = i * b - lo, j * b - lo
            hr, hc = min(b, hi - i * b), min(b, hi - j * b)
            v[:hr, :hc] = Zd[ri:ri + hr, rj:rj + hc]
            if np.any(v):
                out[(i, j)] = v
    return truncate(BM(St.n, b, out), tau)


def irsi(S, tau: float, m: int = 4, start: str = "sqrt2_over_gersh", start_value=None, stop: str = "paper",
         tol: float = 0.0, max_iter: int = 100):
    """IRSI (Sec. 2.2) on a block list: Z_0 = c I, delta_0 = I - c^2 S.
    Returns (Z as BM, RefineInfo, c)."""
    St = truncate(from_blocks(S), tau)
    n, b = St.n, St.b
    if start in ("sqrt2_over_gersh", "inv_sqrt_gersh"):
        rowsum = np.zeros(St.nb * b)
        for (i, _j), v in St.blocks.items():
            rowsum[i * b:(i + 1) * b] += np.sum(np.abs(v), axis=1)
        beta = float(np.max(rowsum[:n]))
        c = math.sqrt(2.0 / beta) if start == "sqrt2_over_gersh" else 1.0 / math.sqrt(beta)
    else:
        c = R.start_scale(None, start, start_value)
    Z0 = identity(n, b, c)
    delta0 = axpy(-c * c, St, 1.0, identity(n, b, 1.0))
    Z, info = localized_refinement(St, Z0, delta0, tau, m, stop, tol, max_iter, 0, St.nb)
    return Z, info, c


def lif(S, tau: float, m: int = 4, base_rows: int = 4096, stop: str = "paper", tol: float = 0.0,
        max_iter: int = 100):
    """LIF (Alg. 2) on a block list, the recursion of ``refinement.lif``.
    Returns (Z as BM, plan with per-node RefineInfo)."""
    St = truncate(from_blocks(S), tau)
    b = St.b
    plan = R.lif_plan(St.n, b, base_rows)

    def rec(node):
        if not node.children:
            return _leaf(St, node.lo, node.hi, tau)
        a, c = node.children
        ZA, ZC = rec(a), rec(c)
        ra0, ra1 = a.lo // b, (a.hi + b - 1) // b
        rc0, rc1 = c.lo // b, (c.hi + b - 1) // b
        B = restrict(St, ra0, ra1, rc0, rc1)
        X = mult(mult(transpose(ZA), B, tau), ZC, tau)
        Z0 = axpy(1.0, ZA, 1.0, ZC)
        delta0 = axpy(-1.0, X, -1.0, transpose(X))
        Sn = restrict(St, ra0, rc1, ra0, rc1)
        node.info = R.RefineInfo()
        Z, info = localized_refinement(Sn, Z0, delta0, tau, m, stop, tol, max_iter, ra0, rc1)
        node.info = info
        return Z

    return rec(plan), plan


def rinch(S, tau: float, base_rows: int = 4096) -> BM:
    """RINCH (Alg. 1) on a block list, the recursion of ``refinement.rinch``."""
    St = truncate(from_blocks(S), tau)
    b = St.b

    def rec(Sn: BM, lo: int, hi: int) -> BM:
        if hi - lo <= base_rows:
            return _leaf(Sn, lo, hi, tau)
        h = lo + R.split_point(hi - lo, b)
        r0, rm, r1 = lo // b, h // b, (hi + b - 1) // b
        Z00 = rec(restrict(Sn, r0, rm, r0, rm), lo, h)
        R_ = mult(transpose(Z00), restrict(Sn, r0, rm, rm, r1), tau)
        Q = axpy(1.0, restrict(Sn, rm, r1, rm, r1), -1.0, mult(transpose(R_), R_, tau))
        Z11 = rec(Q, h, hi)
        Z01 = mult(mult(Z00, R_, tau), Z11, tau)
        return axpy(1.0, axpy(1.0, Z00, -1.0, Z01), 1.0, Z11)

    return rec(St, 0, St.n)
