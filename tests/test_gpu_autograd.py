"""The torch.autograd.Function of the binding (LIFFunction) and factorize():
forward through lif_localized / lif_refine, backward through lif_backward.

Checks: Z equals the handle's result bitwise; S_vals.grad equals the
handle's lif_backward on the same G bitwise (the same library call); a
central difference of the loss along a symmetric direction matches
<grad, E> (h = 1e-6, FP64: ~1e-6 relative at tau = 0; at tau > 0 only to
the effect of the truncation, which the adjoint does not differentiate);
blocks of S removed by the truncation get a zero gradient.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gen import BlockMatrix, overlap_blocks, random_symmetric_on_pattern, water_cluster  # noqa: E402
from paper_1901_07993_amd import lif  # noqa: E402

from test_gpu_parity import dev  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pattern(S):
    return lif.DeviceBlocks(S.n, S.b, torch.from_numpy(S.brow).cuda(), torch.from_numpy(S.bcol).cuda(), None)


@pytest.mark.parametrize("method,opts,tau", [("lif", {"base_rows": 160}, 0.0), ("irsi", {}, 0.0),
                                             ("lif", {"base_rows": 160}, 1e-6)])
def test_lif_function_gradient(method, opts, tau):
    c_, e_ = water_cluster(40, 13)
    S = overlap_blocks(c_, e_, 32)                 # n = 280, b = 32, ragged last block
    opts = dict(opts, tau=tau)
    say(f"case LIFFunction {method} tau={tau}")
    pat = _pattern(S)
    S_vals = torch.from_numpy(S.vals).cuda().requires_grad_(True)
    Z_vals, zr, zc = lif.LIFFunction.apply(S_vals, pat, method, opts)
    gen = torch.Generator().manual_seed(1003)
    Gt = torch.randn(Z_vals.shape, generator=gen, dtype=torch.float64).cuda()
    loss = (Gt * Z_vals).sum()
    loss.backward()
    grad = S_vals.grad.cpu().numpy()

    # the same library calls through the handle (G without Z's padding,
    # whose entries are constant zeros)
    Gh = Gt.cpu().numpy().copy()
    nb = (S.n + S.b - 1) // S.b
    tail = S.n - (nb - 1) * S.b
    Gh[zr.cpu().numpy() == nb - 1, tail:, :] = 0.0
    Gh[zc.cpu().numpy() == nb - 1, :, tail:] = 0.0
    Gb = BlockMatrix(S.n, S.b, zr.cpu().numpy(), zc.cpu().numpy(), Gh)
    with lif.Factorization(dev(S), checkpoint=1, **opts) as f:
        (f.localized if method == "lif" else f.refine)()
        Zh = f.get_Z()
        dS = f.backward(dev(Gb))
    assert np.array_equal(Zh.brow, zr.cpu().numpy()) and np.array_equal(Zh.vals, Z_vals.detach().cpu().numpy())
    pos = {(int(r), int(c)): k for k, (r, c) in enumerate(zip(S.brow, S.bcol))}
    kept = np.zeros(S.nnzb, bool)
    for k, (r, c) in enumerate(zip(dS.brow, dS.bcol)):
        kept[pos[(int(r), int(c))]] = True
        assert np.array_equal(grad[pos[(int(r), int(c))]], dS.vals[k])
    assert np.all(grad[~kept] == 0.0)
    if tau > 0:
        say(f"  {int((~kept).sum())} of {S.nnzb} blocks of S truncated away")

    # central difference of the loss along a symmetric direction of S's kept blocks
    E = random_symmetric_on_pattern(S, 2000)
    E.vals[~kept] = 0.0
    h = 1e-6
    with torch.no_grad():
        lp = (Gt * lif.LIFFunction.apply(S_vals + h * torch.from_numpy(E.vals).cuda(), pat, method, opts)[0]).sum()
        lm = (Gt * lif.LIFFunction.apply(S_vals - h * torch.from_numpy(E.vals).cuda(), pat, method, opts)[0]).sum()
    fd = float(lp - lm) / (2 * h)
    an = float(np.sum(grad * E.vals))
    say(f"  <grad, E> {an:.10e} central difference {fd:.10e}")
    # at tau > 0 the forward truncates blocks while the adjoint differentiates
    # the untruncated recurrence (frozen iteration counts), so the two agree
    # only to the truncation's effect (2e-4 relative observed at tau = 1e-6)
    assert abs(fd - an) <= (1e-5 if tau == 0.0 else 2e-3) * abs(an) + 1e-9


def test_factorize_host_and_device():
    c_, e_ = water_cluster(20, 3)
    S = overlap_blocks(c_, e_, 32)
    say("case factorize host/device")
    Zh, ih = lif.factorize(S, "lif", base_rows=64)
    Zd, idv = lif.factorize(dev(S), "lif", base_rows=64)
    assert isinstance(Zh, lif.HostBlocks) and isinstance(Zd, lif.DeviceBlocks)
    assert np.array_equal(Zh.vals, Zd.vals.cpu().numpy()) and ih["iterations_top"] == idv["iterations_top"]
    Zr, _ = lif.factorize(S, "rinch", base_rows=64)
    Zi, _ = lif.factorize(S, "irsi")
    assert Zr.nnzb > 0 and Zi.nnzb > 0
