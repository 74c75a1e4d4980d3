"""GPU tests of lif_residual_against (Table 1's residual against a matrix other
than the handle's truncated S) and lif_set_opts (one handle, several runs).

* Against the handle's own S the residual is the same computation as
  lif_residual, so the two agree to the last bit; against the matrix before
  the block truncation it matches the oracle's untruncated FP64 residual of
  the same Z (dense, summation order only: 1e-10 relative).
* A handle whose options were changed runs exactly what a new handle with
  those options runs: Z bit for bit.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gen import blocks_to_dense, overlap_blocks, water_cluster  # noqa: E402
from oracle import refinement as R  # noqa: E402
from paper_1901_07993_amd import lif  # noqa: E402

from test_gpu_parity import dev  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_residual_against_truncated_and_untruncated_s():
    c_, e_ = water_cluster(120, 21)
    S = overlap_blocks(c_, e_, 32)                 # n = 840, b = 32, 27 block rows (ragged)
    tau = 1e-5
    say(f"case residual against, n={S.n}, tau={tau}")
    with lif.Factorization(dev(S), tau=tau, base_rows=256) as f:
        f.localized()
        Z = f.get_Z()
        own = f.residual()
        untr = f.residual_against(dev(S))          # S before the block truncation
        untr_host = f.residual_against(S)
    D = blocks_to_dense(S)
    Dt = R.truncate(D, 32, tau)
    Zd = blocks_to_dense(Z)
    ref_t = R.true_residual(Dt, Zd)
    ref_u = R.true_residual(D, Zd)
    say(f"  truncated S: {own:.6e} (oracle {ref_t:.6e}); untruncated S: {untr:.6e} (oracle {ref_u:.6e})")
    assert np.count_nonzero(D != Dt) > 0, "the threshold must remove blocks"
    assert abs(own - ref_t) <= 1e-10 * ref_t
    assert abs(untr - ref_u) <= 1e-10 * ref_u
    assert untr == untr_host
    assert untr != own


def test_residual_against_own_s_is_lif_residual():
    c_, e_ = water_cluster(60, 22)
    S = overlap_blocks(c_, e_, 64)                 # n = 420, b = 64, tau = 0: S is kept whole
    with lif.Factorization(dev(S)) as f:
        f.refine()
        assert f.residual() == f.residual_against(dev(S))


def test_set_opts_runs_as_a_new_handle():
    c_, e_ = water_cluster(150, 23)
    S = overlap_blocks(c_, e_, 64)
    say(f"case set_opts, n={S.n}")
    kw = dict(tau=1e-8, base_rows=320)
    with lif.Factorization(dev(S), **kw) as f:
        i64 = f.localized()
        f.set_opts(prec=lif.MIXED_BF16, prec_switch=1e-2, sym_delta=1)
        ib = f.localized()
        Zb = f.get_Z()
        f.set_opts(prec=lif.FP64, prec_switch=0.0, sym_delta=0)
        i64b = f.localized()
        Z64b = f.get_Z()
    with lif.Factorization(dev(S), prec=lif.MIXED_BF16, prec_switch=1e-2, sym_delta=1, **kw) as g:
        jb = g.localized()
        Zg = g.get_Z()
    with lif.Factorization(dev(S), **kw) as g:
        g.localized()
        Z64 = g.get_Z()
    assert ib["iterations_reduced"] == jb["iterations_reduced"] > 0
    assert i64["iterations_total"] == i64b["iterations_total"]
    for A, B in ((Zb, Zg), (Z64b, Z64)):
        assert np.array_equal(A.brow, B.brow) and np.array_equal(A.bcol, B.bcol)
        assert np.array_equal(A.vals, B.vals)
    # tau and the cap belong to the handle
    with lif.Factorization(dev(S), **kw) as f:
        for bad in (dict(tau=1e-6), dict(mem_cap_bytes=1 << 30), dict(m=0)):
            with pytest.raises(lif.LifError) as ei:
                f.set_opts(**bad)
            assert ei.value.status == lif.ERR_INVALID
