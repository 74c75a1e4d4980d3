"""The allocation-free product lif_multiply_noalloc, through the C ABI,
against the handle-based lif_multiply / lif_multiply_add on the same inputs:
the same kernels run in the same order, so pattern and values must agree bit
for bit.  Two calls in a row, the second on a smaller input with another
block size (the scratch array keeps the first call's contents), a reduced
precision call with an added term, a short output capacity and a product too
large for the scratch array (both rejected with their status, and the array
still usable afterwards)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gen import blocks_to_dense  # noqa: E402
from oracle.blocks import product_count  # noqa: E402
from paper_1901_07993_amd import lif  # noqa: E402

from test_gpu_parity import dev, identity_blocks, random_block_sparse  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def host(C):
    return (C.brow.cpu().numpy(), C.bcol.cpu().numpy(), C.vals.cpu().numpy())


def same(C_dev, C_host):
    r, c, v = host(C_dev)
    return (np.array_equal(r, C_host.brow) and np.array_equal(c, C_host.bcol)
            and np.array_equal(v, C_host.vals))


def handle_product(A, ta, B, tb, tau, prec=lif.FP64, alpha=1.0, D=None, gamma=0.0, upper=False):
    with lif.Factorization(identity_blocks(A.n, A.b), prec=prec) as f:
        return f.multiply(dev(A), ta, dev(B), tb, tau, upper=upper, alpha=alpha, D=None if D is None else dev(D),
                          gamma=gamma)


def test_noalloc_matches_handle_product_twice():
    # call 1: n = 2577 (41 block rows of 64, ragged), truncated
    n1, b1 = 64 * 40 + 17, 64
    A = random_block_sparse(n1, b1, 0.3, 41, scale_spread=3.0)
    B = random_block_sparse(n1, b1, 0.3, 42, scale_spread=3.0)
    D1 = blocks_to_dense(A) @ blocks_to_dense(B)
    tau = float(np.median(np.abs(D1[D1 != 0]))) * 8
    say(f"case noalloc call 1 n={n1} b={b1} tau={tau:.3e}")
    C, p = lif.multiply_noalloc(dev(A), False, dev(B), True, tau)
    R, pr = handle_product(A, False, B, True, tau)
    assert p == pr == product_count(A, False, B, True)
    assert same(C, R) and R.nnzb > 0
    # call 2: smaller, another block size, transposed A
    n2, b2 = 32 * 15 + 5, 32
    A2 = random_block_sparse(n2, b2, 0.5, 43)
    B2 = random_block_sparse(n2, b2, 0.5, 44)
    say(f"case noalloc call 2 n={n2} b={b2}")
    C2, p2 = lif.multiply_noalloc(dev(A2), True, dev(B2), False, 0.0)
    R2, pr2 = handle_product(A2, True, B2, False, 0.0)
    assert p2 == pr2 == product_count(A2, True, B2, False)
    assert same(C2, R2)
    ref = blocks_to_dense(A2).T @ blocks_to_dense(B2)
    got = blocks_to_dense(lif.HostBlocks(n2, b2, *host(C2)))
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.sqrt(n2) * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("prec", [lif.MIXED_BF16, lif.MIXED_FP32])
def test_noalloc_reduced_precision_with_added_term(prec):
    n, b = 64 * 9 + 33, 64
    A = random_block_sparse(n, b, 0.4, 51)
    B = random_block_sparse(n, b, 0.4, 52)
    D = random_block_sparse(n, b, 0.3, 53)
    say(f"case noalloc reduced prec={prec} n={n}")
    C, p = lif.multiply_noalloc(dev(A), False, dev(B), False, 0.0, prec=prec, alpha=0.2734375, D=dev(D),
                                gamma=0.3125)
    R, pr = handle_product(A, False, B, False, 0.0, prec=prec, alpha=0.2734375, D=D, gamma=0.3125)
    assert p == pr
    assert same(C, R)


def test_noalloc_upper_triangle():
    n, b = 32 * 12 + 7, 32
    A = random_block_sparse(n, b, 0.4, 61)
    say(f"case noalloc upper n={n}")
    C, _ = lif.multiply_noalloc(dev(A), True, dev(A), False, 0.0, upper=True)
    R, _ = handle_product(A, True, A, False, 0.0, upper=True)
    assert same(C, R)
    assert np.all(C.bcol.cpu().numpy() >= C.brow.cpu().numpy())


def test_noalloc_rejects_short_capacity_and_oversized_products():
    n, b = 32 * 10 + 3, 32
    A = random_block_sparse(n, b, 0.5, 71)
    B = random_block_sparse(n, b, 0.5, 72)
    R, _ = handle_product(A, False, B, False, 0.0)
    say("case noalloc short capacity")
    with pytest.raises(lif.LifError) as ei:
        lif.multiply_noalloc(dev(A), False, dev(B), False, 0.0, capacity=R.nnzb - 1)
    assert ei.value.status == lif.ERR_INVALID and ei.value.nnzb == R.nnzb
    # 100 x 100 dense blocks of 64: 312 MiB of output values alone
    nb = 100
    say("case noalloc oversized product")
    full = lif.DeviceBlocks(nb * 64, 64,
                            torch.arange(nb, dtype=torch.int32, device="cuda").repeat_interleave(nb),
                            torch.arange(nb, dtype=torch.int32, device="cuda").repeat(nb),
                            torch.full((nb * nb, 64, 64), 1e-3, dtype=torch.float64, device="cuda"))
    with pytest.raises(lif.LifError) as ei:
        lif.multiply_noalloc(full, False, full, False, 0.0, capacity=0)
    assert ei.value.status == lif.ERR_OUT_OF_MEMORY
    assert "scratch" in str(ei.value) and "256 MiB" in str(ei.value)
    del full
    # the array is usable again, and the result matches the handle's
    C, _ = lif.multiply_noalloc(dev(A), False, dev(B), False, 0.0)
    assert same(C, R)
