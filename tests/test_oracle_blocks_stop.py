"""Pins of the oracle's block-product helpers and of its stopping rule.

``oracle.blocks.product_block`` / ``product_count`` are the checkers behind the
full-size sampled-block and exact-count GPU assertions.  They are pinned here
against a dense numpy product of the same block lists (the definition of the
block-sparse product of Sec. 4: block (i, j) of op(A) op(B) is the (i, j) tile
of the dense product) and against a brute-force count over every (i, k, j)
triple, in all four transpose combinations, with non-symmetric blocks and
patterns and a ragged last block.

``oracle.refinement.stop_now`` is pinned on hand-built norm sequences that
tell the exponent m + 1 of Sec. 2.2 from m and m + 2, that fix the first
comparison at k = 2, that stop on delta_k = 0, and that cover the tolerance
rule and its stagnation branch.  A refinement whose delta_0 is already small
pins the driver's use of the rule: delta_0 never enters the comparison, so
two iterations run.

Each group ends with planted mistakes that these pins must reject.
"""
import itertools

import numpy as np
import pytest

import oracle.refinement as R
from gen import BlockMatrix, blocks_to_dense, dense_to_blocks
from oracle.blocks import BlockDict, product_block, product_count


def _random_blocks(n, b, density, seed):
    """Non-symmetric block-sparse matrix: independent pattern and values."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nb = (n + b - 1) // b
    mask = rng.random((nb, nb)) < density
    mask[0, nb - 1] = True          # make sure the ragged corner takes part
    mask[nb - 1, 0] = False
    A = rng.standard_normal((nb * b, nb * b))
    A *= np.repeat(np.repeat(mask, b, 0), b, 1)
    return dense_to_blocks(A[:n, :n], b)


def _cases():
    # (n, b): several blocks and a ragged tail
    for n, b in ((5 * 8 + 3, 8), (4 * 16 + 15, 16)):
        A = _random_blocks(n, b, 0.45, 100 + n)
        B = _random_blocks(n, b, 0.4, 200 + n)
        yield A, B


def _brute_count(A, ta, B, tb):
    """Number of triples (i, k, j) with op(A)_ik and op(B)_kj both stored."""
    pa = {(int(c), int(r)) if ta else (int(r), int(c)) for r, c in zip(A.brow, A.bcol)}
    pb = {(int(c), int(r)) if tb else (int(r), int(c)) for r, c in zip(B.brow, B.bcol)}
    nb = A.nb
    return sum(1 for i, k, j in itertools.product(range(nb), repeat=3) if (i, k) in pa and (k, j) in pb)


def _check_product_block(fn):
    """True when ``fn`` reproduces every block of the dense product and the
    number of contributing inner indices, in all four transposes."""
    for A, B in _cases():
        b, nb = A.b, A.nb
        Da, Db = blocks_to_dense(A), blocks_to_dense(B)
        pa = {(int(r), int(c)) for r, c in zip(A.brow, A.bcol)}
        pb = {(int(r), int(c)) for r, c in zip(B.brow, B.bcol)}
        da, db = BlockDict(A), BlockDict(B)
        for ta, tb in itertools.product((False, True), repeat=2):
            full = (Da.T if ta else Da) @ (Db.T if tb else Db)
            P = np.zeros((nb * b, nb * b))
            P[:A.n, :A.n] = full
            for i in range(nb):
                for j in range(nb):
                    blk, cnt = fn(da, ta, db, tb, i, j)
                    ks = [k for k in range(nb)
                          if ((k, i) if ta else (i, k)) in pa and ((j, k) if tb else (k, j)) in pb]
                    if cnt != len(ks):
                        return False
                    ref = P[i * b:(i + 1) * b, j * b:(j + 1) * b]
                    if not ks:
                        if blk is not None:
                            return False
                        continue
                    if np.max(np.abs(blk - ref)) > 1e-12 * max(1.0, np.max(np.abs(ref))):
                        return False
    return True


def _check_product_count(fn):
    for A, B in _cases():
        for ta, tb in itertools.product((False, True), repeat=2):
            if fn(A, ta, B, tb) != _brute_count(A, ta, B, tb):
                return False
    return True


def test_product_block_matches_dense_product():
    assert _check_product_block(product_block)


def test_product_count_matches_brute_force():
    assert _check_product_count(product_count)


def test_product_count_examples_by_hand():
    # A = [[x, x], [0, x]] (blocks (0,0), (0,1), (1,1)), B = A:
    # row 0 of A meets rows 0 (2 blocks) and 1 (1 block) of B -> 3, row 1 -> 1
    b = 2
    vals = np.ones((3, b, b))
    A = BlockMatrix(4, b, np.array([0, 0, 1], np.int32), np.array([0, 1, 1], np.int32), vals)
    assert product_count(A, False, A, False) == 4
    # A^T A: rows of A^T are columns of A: column 0 holds (0,0) -> meets row 0 of A (2);
    # column 1 holds (0,1), (1,1) -> rows 0 and 1 of A (2 + 1)
    assert product_count(A, True, A, False) == 5
    # A A^T: row 0 of A meets rows 0, 1 of A^T = columns 0, 1 of A (1 + 2), row 1 meets column 1 (2)
    assert product_count(A, False, A, True) == 5


# --- planted mistakes in the block helpers ---------------------------------

def test_planted_untransposed_column_block_is_caught():
    def bad(A, ta, B, tb, i, j):
        ra = A.op_row(i, ta)
        cb = B.cols.get(j, {}) if not tb else dict(B.rows.get(j, {}))  # forgot the block transpose
        ks = sorted(set(ra) & set(cb))
        if not ks:
            return None, 0
        acc = np.zeros((A.b, A.b))
        for k in ks:
            acc += ra[k] @ cb[k]
        return acc, len(ks)
    assert not _check_product_block(bad)


def test_planted_swapped_operands_are_caught():
    def bad(A, ta, B, tb, i, j):
        ra = A.op_row(i, ta)
        cb = B.op_col(j, tb)
        ks = sorted(set(ra) & set(cb))
        if not ks:
            return None, 0
        acc = np.zeros((A.b, A.b))
        for k in ks:
            acc += cb[k] @ ra[k]
        return acc, len(ks)
    assert not _check_product_block(bad)


def test_planted_count_ignoring_transpose_is_caught():
    def bad(A, ta, B, tb):
        ac = np.asarray(A.brow) if ta else np.asarray(A.bcol)
        br = np.asarray(B.brow)              # ignores tb
        row_len_b = np.bincount(br, minlength=A.nb)
        return int(row_len_b[ac].sum())
    assert not _check_product_count(bad)


def test_planted_count_wrong_inner_index_is_caught():
    def bad(A, ta, B, tb):
        ac = np.asarray(A.bcol) if ta else np.asarray(A.brow)  # output row taken as inner index
        br = np.asarray(B.bcol) if tb else np.asarray(B.brow)
        row_len_b = np.bincount(br, minlength=A.nb)
        return int(row_len_b[ac].sum())
    assert not _check_product_count(bad)


# ----------------------------------------------------------------------------
# stopping rule
# ----------------------------------------------------------------------------

def _paper_stops(fn, m=4):
    """The hand-built decisions of the paper's rule: ||delta_k|| > ||delta_{k-1}||^{m+1}."""
    ok = True
    e_prev = 0.1
    # m = 4: e_prev^5 = 1e-5, e_prev^4 = 1e-4, e_prev^6 = 1e-6
    ok &= fn(2, 5e-5, e_prev, m, "paper", 0.0) is True     # above e^{m+1}, below e^m
    ok &= fn(2, 5e-6, e_prev, m, "paper", 0.0) is False    # below e^{m+1}, above e^{m+2}
    ok &= fn(2, 2e-4, e_prev, m, "paper", 0.0) is True     # above both
    ok &= fn(3, 1e-7, e_prev, m, "paper", 0.0) is False    # below both
    # m = 2: e_prev^3 = 1e-3
    ok &= fn(2, 2e-3, e_prev, 2, "paper", 0.0) is True
    ok &= fn(2, 5e-4, e_prev, 2, "paper", 0.0) is False
    # equality does not stop (strict comparison)
    ok &= fn(2, 0.5 ** 5, 0.5, 4, "paper", 0.0) is False
    # first iteration: nothing to compare with, only delta_1 = 0 stops
    ok &= fn(1, 0.7, None, m, "paper", 0.0) is False
    ok &= fn(1, 1e-300, None, m, "paper", 0.0) is False
    ok &= fn(1, 0.0, None, m, "paper", 0.0) is True
    ok &= fn(4, 0.0, 1e-3, m, "paper", 0.0) is True
    return bool(ok)


def _tol_stops(fn):
    ok = True
    ok &= fn(3, 1e-11, 1e-6, 4, "tol", 1e-10) is True      # reached
    ok &= fn(3, 1e-10, 1e-6, 4, "tol", 1e-10) is True      # equality reaches
    ok &= fn(3, 2e-10, 1e-9, 4, "tol", 1e-10) is False     # still decreasing
    ok &= fn(3, 1e-9, 1e-9, 4, "tol", 1e-10) is True       # stagnated (not decreasing)
    ok &= fn(3, 2e-9, 1e-9, 4, "tol", 1e-10) is True       # grew below 1: stagnation, not divergence
    ok &= fn(1, 0.5, None, 4, "tol", 1e-10) is False
    return bool(ok)


def test_paper_rule_exponent_and_first_test():
    assert _paper_stops(R.stop_now)


def test_tol_rule_and_stagnation():
    assert _tol_stops(R.stop_now)


def test_divergence_is_reported():
    with pytest.raises(R.NoConvergence):
        R.stop_now(3, 1.5, 1.2, 4, "paper", 0.0)     # grows while >= 1
    with pytest.raises(R.NoConvergence):
        R.stop_now(3, float("nan"), 0.5, 4, "tol", 1e-10)
    # growth below 1 is the paper rule's stop, not divergence
    assert R.stop_now(3, 0.6, 0.5, 4, "paper", 0.0) is True


def _near_converged_run(m=4):
    """Refinement from a start whose delta_0 has norm ~1e-4: delta_1 lands at
    the rounding floor, far above ||delta_0||^{m+1} ~ 1e-20."""
    rng = np.random.Generator(np.random.PCG64(7))
    n = 48
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.linspace(0.5, 2.0, n)
    S = (Q * lam) @ Q.T
    S = 0.5 * (S + S.T)
    w, V = np.linalg.eigh(S)
    Zex = (V / np.sqrt(w)) @ V.T
    E = rng.standard_normal((n, n))
    Z0 = Zex + 2e-6 * (E + E.T)
    delta0 = np.eye(n) - Z0.T @ S @ Z0
    return S, Z0, delta0


def test_driver_never_compares_with_delta0():
    S, Z0, delta0 = _near_converged_run()
    e0 = float(np.linalg.norm(delta0))
    assert 1e-5 < e0 < 1e-3
    Z, info = R.localized_refinement(S, Z0, delta0, 16, 0.0, m=4, stop="paper")
    # delta_1 is at the rounding floor (> e0^5): a rule that compared it with
    # delta_0 would stop after one iteration; the paper's first test is k = 2
    assert info.norms[0] > e0 ** 5
    assert info.iterations == 2
    assert info.norms[1] > info.norms[0] ** 5


# --- planted mistakes in the stopping rule -----------------------------------

def test_planted_exponent_m_is_caught():
    def bad(k, e, e_prev, m, stop, tol):
        R.check_divergence(k, e, e_prev)
        if e == 0.0:
            return True
        return e_prev is not None and e > e_prev ** m
    assert not _paper_stops(bad)


def test_planted_exponent_m_plus_2_is_caught():
    def bad(k, e, e_prev, m, stop, tol):
        R.check_divergence(k, e, e_prev)
        if e == 0.0:
            return True
        return e_prev is not None and e > e_prev ** (m + 2)
    assert not _paper_stops(bad)


def test_planted_non_strict_or_missing_zero_test_is_caught():
    def ge(k, e, e_prev, m, stop, tol):
        return e == 0.0 or (e_prev is not None and e >= e_prev ** (m + 1))

    def nozero(k, e, e_prev, m, stop, tol):
        return e_prev is not None and e > e_prev ** (m + 1)
    assert not _paper_stops(ge)
    assert not _paper_stops(nozero)


def test_planted_tol_without_stagnation_is_caught():
    def bad(k, e, e_prev, m, stop, tol):
        return e <= tol
    assert not _tol_stops(bad)


def test_planted_delta0_in_comparison_is_caught(monkeypatch):
    # a driver that seeds the comparison with ||delta_0|| stops after one iteration
    good = R.stop_now
    seen = {}

    def seeded(k, e, e_prev, m, stop, tol):
        if k == 1:
            e_prev = seen["e0"]
        return good(k, e, e_prev, m, stop, tol)

    S, Z0, delta0 = _near_converged_run()
    seen["e0"] = float(np.linalg.norm(delta0))
    monkeypatch.setattr(R, "stop_now", seeded)
    with pytest.raises(AssertionError):
        test_driver_never_compares_with_delta0()
