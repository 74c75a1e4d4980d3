"""Single output blocks of a block-sparse product, for sampled checks at sizes
the dense oracle cannot hold.  Test infrastructure only.

A block list (n, b, brow, bcol, vals) is indexed as a dict; the (i, j) block
of op(A) op(B) is the plain sum over k of op(A)_{ik} op(B)_{kj} (Sec. 4: zero
blocks contribute nothing and are skipped).
"""
from __future__ import annotations

import numpy as np


class BlockDict:
    def __init__(self, M):
        self.b = int(M.b)
        self.rows: dict[int, dict[int, np.ndarray]] = {}
        self.cols: dict[int, dict[int, np.ndarray]] = {}
        for r, c, v in zip(np.asarray(M.brow).tolist(), np.asarray(M.bcol).tolist(), M.vals):
            self.rows.setdefault(r, {})[c] = v
            self.cols.setdefault(c, {})[r] = v

    def op_row(self, i: int, trans: bool) -> dict[int, np.ndarray]:
        """Blocks of row i of op(M): {k: block}."""
        if trans:
            return {k: v.T for k, v in self.cols.get(i, {}).items()}
        return self.rows.get(i, {})

    def op_col(self, j: int, trans: bool) -> dict[int, np.ndarray]:
        """Blocks of column j of op(M): {k: block}."""
        if trans:
            return {k: v.T for k, v in self.rows.get(j, {}).items()}
        return self.cols.get(j, {})


def product_block(A: BlockDict, ta: bool, B: BlockDict, tb: bool, i: int, j: int):
    """(block (i, j) of op(A) op(B) or None if no k contributes, number of k)."""
    ra = A.op_row(i, ta)
    cb = B.op_col(j, tb)
    ks = sorted(set(ra) & set(cb))
    if not ks:
        return None, 0
    acc = np.zeros((A.b, A.b))
    for k in ks:
        acc += ra[k] @ cb[k]
    return acc, len(ks)


def product_count(A, ta: bool, B, tb: bool) -> int:
    """Number of block products sum_i sum_{k in op(A)(i,:)} |op(B)(k,:)| (integer)."""
    ar, ac = (np.asarray(A.bcol), np.asarray(A.brow)) if ta else (np.asarray(A.brow), np.asarray(A.bcol))
    br = np.asarray(B.bcol) if tb else np.asarray(B.brow)
    nb = (int(A.n) + int(A.b) - 1) // int(A.b)
    row_len_b = np.bincount(br, minlength=nb)
    return int(row_len_b[ac].sum())
