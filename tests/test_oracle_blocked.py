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


# ----------------------------------------------------------------------------
# the oracle's C block product (oracle/bsmm.c) against the Python loop and
# dense numpy products
# ----------------------------------------------------------------------------

def _random_bm(n, b, density, seed, spread=3.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    nb = (n + b - 1) // b
    A = OB.BM(n, b)
    for i in range(nb):
        for j in range(nb):
            if rng.random() < density:
                v = rng.standard_normal((b, b)) * 10.0 ** (-spread * rng.random())
                v[max(0, n - i * b):, :] = 0.0
                v[:, max(0, n - j * b):] = 0.0
                A.blocks[(i, j)] = v
    return A


def _check_c_product(mult):
    for n, b, seed in ((7 * 8 + 5, 8, 1), (5 * 32 + 11, 32, 2)):
        A = _random_bm(n, b, 0.45, 10 + seed)
        B = _random_bm(n, b, 0.4, 20 + seed)
        full = OB.to_dense(A) @ OB.to_dense(B)
        nrm = R.block_norms(full, b)
        srt = np.sort(nrm[nrm > 0])
        tau = float(np.sqrt(srt[len(srt) // 2 - 1] * srt[len(srt) // 2]))   # no norm near tau
        for t in (0.0, tau):
            C = mult(A, B, t)
            P = OB.mult_py(A, B, t)
            if set(C.blocks) != set(P.blocks):
                return False
            ref = R.truncate(full, b, t)
            if np.max(np.abs(OB.to_dense(C) - ref)) > 1e-13 * np.max(np.abs(ref)):
                return False
            if max(np.max(np.abs(C.blocks[k] - P.blocks[k])) for k in C.blocks) > 1e-13 * np.max(np.abs(ref)):
                return False
    return True


def test_c_block_product_matches_python_loop_and_dense():
    if OB._clib() is None:
        pytest.skip("oracle/libbsmm.so not built (oracle/build.py)")
    assert _check_c_product(OB.mult)


def test_planted_c_product_layout_mistake_is_caught(monkeypatch):
    if OB._clib() is None:
        pytest.skip("oracle/libbsmm.so not built (oracle/build.py)")
    good = OB._csr

    def transposed_blocks(A):
        rp, cols, vals = good(A)
        return rp, cols, np.ascontiguousarray(vals.transpose(0, 2, 1))
    monkeypatch.setattr(OB, "_csr", transposed_blocks)
    assert not _check_c_product(OB.mult)
