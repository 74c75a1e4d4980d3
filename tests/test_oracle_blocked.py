"""Pins of the block-sparse oracle (oracle/blocked.py) to the dense oracle,
which the closed forms pin: on inputs both can run, at tau = 0 and tau > 0,
with a ragged last block, the two give the same iteration counts (per LIF
node) and factors equal up to the summation order inside products."""
import numpy as np
import pytest

import oracle.blocked as OB
import oracle.refinement as R
from gen import blocks_to_dense, config_matrix, overlap_blocks, water_cluster


def rel(A, B):
    return np.linalg.norm(A - B) / np.linalg.norm(B)


def node_iterations(plan):
    out = []

    def walk(nd):
        if nd.children:
            out.append((nd.lo, nd.hi, nd.info.iterations))
            walk(nd.children[0])
            walk(nd.children[1])

    walk(plan)
    return out


def test_blocked_irsi_matches_dense():
    S, _ = config_matrix(0, count=60)      # n = 420, b = 32: ragged last block
    D = blocks_to_dense(S)
    for tau in (0.0, 1e-5):
        Zb, ib, cb = OB.irsi(S, tau)
        Zd, idd, cd = R.irsi(D, 32, tau)
        assert ib.iterations == idd.iterations and cb == cd
        assert np.allclose(ib.norms, idd.norms, rtol=1e-9, atol=1e-14)
        assert rel(OB.to_dense(Zb), Zd) <= 1e-12


@pytest.mark.parametrize("tau", [0.0, 1e-6])
def test_blocked_lif_and_rinch_match_dense(tau):
    c_, e_ = water_cluster(60, 6)
    S = overlap_blocks(c_, e_, 32)        # n = 420
    D = blocks_to_dense(S)
    Zb, pb = OB.lif(S, tau, base_rows=128)
    Zd, pd = R.lif(D, 32, tau, base_rows=128)
    assert node_iterations(pb) == node_iterations(pd)
    assert rel(OB.to_dense(Zb), Zd) <= 1e-12
    assert rel(OB.to_dense(OB.rinch(S, tau, base_rows=128)), R.rinch(D, 32, tau, base_rows=128)) <= 1e-12


def test_blocked_lif_chain_matches_dense():
    S, cfg = config_matrix(1, count=60)    # n = 1200, b = 64, tau = 1e-10
    D = blocks_to_dense(S)
    Zb, pb = OB.lif(S, cfg["tau"], base_rows=256)
    Zd, pd = R.lif(D, 64, cfg["tau"], base_rows=256)
    assert node_iterations(pb) == node_iterations(pd)
    assert rel(OB.to_dense(Zb), Zd) <= 1e-12
    # the block list round trip and the blockwise helpers
    brow, bcol, vals = OB.to_arrays(Zb)
    assert np.all(np.diff(brow.astype(np.int64) * Zb.nb + bcol) > 0)
    assert np.array_equal(OB.to_dense(OB.transpose(Zb)), OB.to_dense(Zb).T)
    I = OB.identity(S.n, 64, 2.0)
    assert np.array_equal(OB.to_dense(I), 2.0 * np.eye(S.n))
