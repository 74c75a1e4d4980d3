"""Synthetic input generator: structure, determinism and padding."""
import numpy as np
import pytest

from gen import (blocks_to_dense, config_matrix, dense_to_blocks, helix_chain, overlap_blocks,
                 random_on_pattern, random_symmetric_on_pattern, water_cluster)
from gen.overlap import _morton_order


def test_water_small_is_spd_unit_diagonal():
    S, cfg = config_matrix(0)
    assert S.n == 700 and S.b == 32 and S.nb == 22
    D = blocks_to_dense(S)
    assert np.array_equal(D, D.T)
    assert np.all(np.diag(D) == 1.0)
    ev = np.linalg.eigvalsh(D)
    assert ev[0] > 1e-3 and ev[-1] / ev[0] < 2e3


def test_block_list_sorted_unique_and_padded():
    c, e = water_cluster(20, 7)          # n = 140, b = 32 -> last block has 12 rows
    S = overlap_blocks(c, e, 32)
    key = S.brow.astype(np.int64) * S.nb + S.bcol
    assert np.all(np.diff(key) > 0)
    tail = S.n - (S.nb - 1) * S.b
    assert tail == 12
    last_r = S.vals[S.brow == S.nb - 1]
    last_c = S.vals[S.bcol == S.nb - 1]
    assert np.all(last_r[:, tail:, :] == 0) and np.all(last_c[:, :, tail:] == 0)
    # symmetric pattern stored in full
    pat = set(zip(S.brow.tolist(), S.bcol.tolist()))
    assert all((c_, r_) in pat for r_, c_ in pat)


def test_seeded_reproducible():
    a = config_matrix(0)[0]
    b = config_matrix(0)[0]
    assert np.array_equal(a.vals, b.vals) and np.array_equal(a.brow, b.brow)
    c = config_matrix(0, count=100)[0]
    assert np.array_equal(a.vals, c.vals)


def test_morton_order_monotone():
    rng = np.random.default_rng(0)
    p = rng.random((500, 3))
    order = _morton_order(p)
    # a Morton order is a permutation and keeps points of one octant together
    assert sorted(order.tolist()) == list(range(500))
    span = float(np.max(p.max(0) - p.min(0)))
    oct_ = ((p[order] >= p.min(0) + span / 2) * np.array([1, 2, 4])).sum(1)
    assert np.all(np.diff(oct_) >= 0)


def test_chain_geometry_and_sparsity():
    c, e = helix_chain(60, 1)
    assert c.shape == (1200, 3)
    d = np.sqrt(((c[:, None] - c[None]) ** 2).sum(-1)) / 1.8897261254578281
    np.fill_diagonal(d, 10.0)
    assert d.min() >= 1.0 - 1e-9
    S = overlap_blocks(c, e, 64, 1e-3 * 1e-10 / 64)
    D = blocks_to_dense(S)
    assert np.allclose(D, D.T)
    assert np.linalg.eigvalsh(D)[0] > 1e-2


def test_dense_roundtrip_and_random_patterns():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((70, 70))
    A[:, 40:64] = 0
    A[40:64, :] = 0
    B = dense_to_blocks(A, 16)
    assert np.array_equal(blocks_to_dense(B), A)
    G = random_on_pattern(B, 3)
    assert G.vals.shape == B.vals.shape
    Sym = dense_to_blocks(A + A.T, 16)
    E = random_symmetric_on_pattern(Sym, 4)
    DE = blocks_to_dense(E)
    assert np.allclose(DE, DE.T) and abs(np.linalg.norm(DE) - 1) < 1e-12
