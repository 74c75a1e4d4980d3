"""GPU parity of the differentiation form: lif_backward against the oracle's
reverse sweep (same frozen iteration counts), the eigendecomposition
references of the converged maps, and central finite differences of the GPU
forward itself.

Tolerances: the GPU and the oracle reverse the same recurrence from iterates
that agree to ~1e-13, so dS agrees to 1e-9 of its largest entry.  Against the
exact-limit references the difference is O(||delta_final||) (1e-13 here).
Finite differences (h = 1e-6, FP64) resolve a directional derivative to about
1e-6 of its size.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gen import BlockMatrix, blocks_to_dense, config_matrix, overlap_blocks, random_on_pattern, \
    random_symmetric_on_pattern, water_cluster  # noqa: E402
from oracle import adjoint as ADJ  # noqa: E402
from oracle import refinement as R  # noqa: E402
from paper_1901_07993_amd import lif  # noqa: E402

from test_gpu_parity import dev  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def on_pattern(D, P):
    """Dense D restricted to the block pattern of P (zero elsewhere)."""
    b = P.b
    nb = P.nb
    mask = np.zeros((nb, nb), bool)
    mask[P.brow, P.bcol] = True
    M = np.repeat(np.repeat(mask, b, 0), b, 1)[:P.n, :P.n]
    return np.where(M, D, 0.0)


def gpu_loss(S, G, E, h, **opts):
    """L(S + h E) with the GPU forward (dense E added on S's pattern)."""
    Sp = BlockMatrix(S.n, S.b, S.brow, S.bcol, S.vals + h * E.vals)
    with lif.Factorization(dev(Sp), **opts) as f:
        if opts.get("base_rows"):
            f.localized()
        else:
            f.refine()
        Z = blocks_to_dense(f.get_Z())
    return float(np.sum(blocks_to_dense(G) * Z))


def test_irsi_backward_matches_oracle_and_references():
    c_, e_ = water_cluster(40, 13)
    S = overlap_blocks(c_, e_, 32)                 # n = 280
    D = blocks_to_dense(S)
    lam = float(np.linalg.eigvalsh(D)[-1])
    G = random_on_pattern(S, 1003)
    Gd = blocks_to_dense(G)
    say("case irsi backward water-40 n=280 b=32")
    opts = dict(start=lif.START_INV_SQRT_LMAX, start_value=lam, checkpoint=1)
    with lif.Factorization(dev(S), **opts) as f:
        info = f.refine()
        dS = f.backward(dev(G))
    K = info["iterations_top"]
    c = 1.0 / np.sqrt(lam)
    got = blocks_to_dense(dS)
    assert np.array_equal(dS.brow, S.brow) and np.array_equal(dS.bcol, S.bcol)
    ref = on_pattern(ADJ.irsi_grad(D, Gd, c, 4, K), S)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= 1e-9 * scale
    lim = on_pattern(ADJ.inv_sqrt_grad(D, Gd), S)
    assert np.max(np.abs(got - lim)) <= 1e-8 * scale
    # central differences of the GPU forward along symmetric directions on S's pattern
    for j in range(2):
        E = random_symmetric_on_pattern(S, 2000 + j)
        h = 1e-6
        fd = (gpu_loss(S, G, E, h, **opts) - gpu_loss(S, G, E, -h, **opts)) / (2 * h)
        an = float(np.sum(got * blocks_to_dense(E)))
        assert abs(fd - an) <= 1e-5 * abs(an) + 1e-9


@pytest.mark.parametrize("b,n_mol,base", [(64, 150, 320), (32, 80, 160)])
def test_lif_backward_matches_oracle_and_references(b, n_mol, base):
    c_, e_ = water_cluster(n_mol, 14)
    S = overlap_blocks(c_, e_, b)
    D = blocks_to_dense(S)
    G = random_on_pattern(S, 1003)
    Gd = blocks_to_dense(G)
    say(f"case lif backward water-{n_mol} n={S.n} b={b} base={base}")
    opts = dict(base_rows=base, checkpoint=1)
    with lif.Factorization(dev(S), **opts) as f:
        info = f.localized()
        dS = f.backward(dev(G))
    got = blocks_to_dense(dS)
    Zo, plan = R.lif(D, b, 0.0, base_rows=base)
    iters = {}

    def walk(nd):
        if nd.children:
            iters[(nd.lo, nd.hi)] = nd.info.iterations
            walk(nd.children[0])
            walk(nd.children[1])

    walk(plan)
    assert info["iterations_top"] == plan.info.iterations
    ref = on_pattern(ADJ.lif_grad(D, Gd, b, base, 4, iters), S)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= 1e-9 * scale
    lim = on_pattern(ADJ.lif_limit_grad(D, Gd, b, base), S)
    assert np.max(np.abs(got - lim)) <= 1e-8 * scale
    E = random_symmetric_on_pattern(S, 2100)
    h = 1e-6
    fd = (gpu_loss(S, G, E, h, **opts) - gpu_loss(S, G, E, -h, **opts)) / (2 * h)
    an = float(np.sum(got * blocks_to_dense(E)))
    assert abs(fd - an) <= 1e-5 * abs(an) + 1e-9


def test_backward_needs_checkpoints():
    S, _ = config_matrix(0, count=20)
    G = random_on_pattern(S, 1)
    say("case backward without checkpoints")
    with lif.Factorization(dev(S)) as f:
        f.refine()
        with pytest.raises(lif.LifError) as ei:
            f.backward(dev(G))
    assert ei.value.status == lif.ERR_STATE
