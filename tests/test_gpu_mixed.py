"""GPU parity of the precision form: products with FP32 / BF16 inputs and FP32
accumulation, and refinement that wins the accuracy back (FP64 delta).

Tolerances, derived from the arithmetic:
* one product: the GPU rounds its inputs exactly as the oracle does (round to
  nearest even; BF16 through FP32), so the only difference is the FP32
  accumulation of K = n terms per entry: |C_gpu - C_oracle| <= n 2^-24 (|A_r||B_r|)
  entrywise, A_r, B_r the rounded inputs;
* a product with an added term (the fused Horner step alpha A B + gamma D):
  the same accumulation bound for the product, plus FP64 rounding of the
  scaling and of the addition; D itself is never rounded;
* refinement: the residual is gated (tracked ||delta||_F <= tol, and the
  untruncated residual agrees with it).  Z is compared with the oracle's
  refinement in the same precision, which reads a Horner factor T = X + c I
  as the device does (only delta and X rounded, c delta added in FP64): both
  sides then round the same values, and they differ only through the FP32
  accumulation of each product, so ||Z - Z_oracle||_F <= n 2^-24 ||Z_oracle||_F
  (the worst-case relative accumulation error of one product of inner length
  n; the refinement does not amplify it, measured 1e-8 to 3e-6).  Against
  the FP64 oracle Z is an inverse factor within 10 u_in (u_in = 2^-24 or
  2^-8): inexact corrections move Z along the set of inverse factors.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gen import blocks_to_dense, config_matrix, overlap_blocks, water_cluster  # noqa: E402
from oracle import refinement as R  # noqa: E402
from oracle.blocks import product_count  # noqa: E402
from paper_1901_07993_amd import lif  # noqa: E402

from test_gpu_parity import dev, identity_blocks, random_block_sparse  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")]

PREC = {"fp32": lif.MIXED_FP32, "bf16": lif.MIXED_BF16}
U_IN = {"fp32": 2.0 ** -24, "bf16": 2.0 ** -8}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(Z, Zref):
    return float(np.linalg.norm(Z - Zref) / np.linalg.norm(Zref))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("b,n", [(32, 200), (64, 300)])
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
def test_mixed_multiply_matches_oracle(prec, b, n, ta, tb):
    say(f"case mixed multiply {prec} b={b} n={n} ta={ta} tb={tb}")
    A = random_block_sparse(n, b, 0.4, 5)
    B = random_block_sparse(n, b, 0.4, 6)
    with lif.Factorization(identity_blocks(n, b), prec=PREC[prec]) as f:
        C, prods = f.multiply(dev(A), ta, dev(B), tb, 0.0)
    Da, Db = blocks_to_dense(A), blocks_to_dense(B)
    Da, Db = (Da.T if ta else Da), (Db.T if tb else Db)
    ref = R.mult(Da, Db, b, 0.0, prec)
    bound = n * 2.0 ** -24 * (np.abs(R.round_to(Da, prec)) @ np.abs(R.round_to(Db, prec))) + 1e-300
    got = blocks_to_dense(C)
    assert prods == product_count(A, ta, B, tb)
    assert np.all(np.abs(got - ref) <= bound)
    # rounding really happened: FP64 differs from the rounded-input product
    assert np.max(np.abs(got - Da @ Db)) > 0


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("b,n", [(32, 200), (64, 300)])
@pytest.mark.parametrize("ta", [False, True])
def test_mixed_multiply_add_matches_oracle(prec, b, n, ta):
    # the fused Horner step: alpha op(A) B + gamma D, with only A and B rounded
    # and D added in FP64 (the oracle's mult_add); D's pattern joins the output
    say(f"case mixed multiply-add {prec} b={b} n={n} ta={ta}")
    A = random_block_sparse(n, b, 0.4, 15)
    B = random_block_sparse(n, b, 0.4, 16)
    D = random_block_sparse(n, b, 0.3, 17)
    alpha, gamma = 0.2734375, 0.3125
    with lif.Factorization(identity_blocks(n, b), prec=PREC[prec]) as f:
        C, prods = f.multiply(dev(A), ta, dev(B), False, 0.0, alpha=alpha, D=dev(D), gamma=gamma)
    Da, Db, Dd = blocks_to_dense(A), blocks_to_dense(B), blocks_to_dense(D)
    Da = Da.T if ta else Da
    ref = R.mult_add(Da, Db, b, 0.0, prec, alpha=alpha, D=Dd, gamma=gamma)
    # FP32 accumulation of n terms, then the FP64 scaling and addition
    bound = (alpha * n * 2.0 ** -24 * (np.abs(R.round_to(Da, prec)) @ np.abs(R.round_to(Db, prec)))
             + 4 * 2.0 ** -53 * (np.abs(ref) + gamma * np.abs(Dd)) + 1e-300)
    got = blocks_to_dense(C)
    assert prods == product_count(A, ta, B, False)
    assert np.all(np.abs(got - ref) <= bound)
    # D is not rounded: where the product has no block, C is exactly gamma D
    prod_pat = (np.abs(Da) @ np.abs(Db)) == 0
    assert np.array_equal(got[prod_pat], (gamma * Dd)[prod_pat])
    # the identity part in the input precision would differ by ~u_in gamma |D|
    worse = R.mult_add(Da, Db, b, 0.0, prec, alpha=alpha, D=R.round_to(Dd, prec), gamma=gamma)
    if prec == "bf16":
        assert np.max(np.abs(worse - ref)) > 100 * np.max(np.abs(got - ref))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mixed_irsi_water100(prec):
    S, _ = config_matrix(0)
    D = blocks_to_dense(S)
    lam = float(np.linalg.eigvalsh(D)[-1])
    say(f"case mixed irsi water-100 {prec}")
    with lif.Factorization(dev(S), prec=PREC[prec], stop=lif.STOP_TOL, tol=1e-10,
                           start=lif.START_INV_SQRT_LMAX, start_value=lam) as f:
        info = f.refine()
        Z = blocks_to_dense(f.get_Z())
        res = f.residual()
    Zm, im, _ = R.irsi(D, 32, 0.0, start="inv_sqrt_lmax", start_value=lam, stop="tol", tol=1e-10, prec=prec)
    Z64, _, _ = R.irsi(D, 32, 0.0, start="inv_sqrt_lmax", start_value=lam, stop="tol", tol=1e-10)
    say(f"  gpu iterations {info['iterations_top']} oracle {im.iterations} norms {info['norms']}")
    assert info["delta_tracked"] <= 1e-10 and not info["stagnated"]
    assert abs(res - info["delta_tracked"]) <= 1e-11
    assert abs(info["iterations_top"] - im.iterations) <= 1
    say(f"  rel diff vs oracle {rel(Z, Zm):.3e}, vs FP64 oracle {rel(Z, Z64):.3e}")
    assert np.linalg.norm(Z - Z64) <= 10 * U_IN[prec] * np.linalg.norm(Z64)
    assert rel(Z, Zm) <= S.n * 2.0 ** -24


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mixed_lif_water(prec):
    c_, e_ = water_cluster(150, 7)
    S = overlap_blocks(c_, e_, 64)
    D = blocks_to_dense(S)
    say(f"case mixed lif water-150 {prec}")
    with lif.Factorization(dev(S), prec=PREC[prec], stop=lif.STOP_TOL, tol=1e-10, base_rows=320) as f:
        info = f.localized()
        Z = blocks_to_dense(f.get_Z())
        res = f.residual()
    Z64, _ = R.lif(D, 64, 0.0, base_rows=320, stop="tol", tol=1e-10)
    Zm, _ = R.lif(D, 64, 0.0, base_rows=320, stop="tol", tol=1e-10, prec=prec)
    say(f"  rel diff vs oracle {rel(Z, Zm):.3e}, vs FP64 oracle {rel(Z, Z64):.3e}")
    assert res <= 1e-10
    assert np.linalg.norm(Z - Z64) <= 10 * U_IN[prec] * np.linalg.norm(Z64)
    assert rel(Z, Zm) <= S.n * 2.0 ** -24


# ----------------------------------------------------------------------------
# precision schedule: reduced precision while ||delta||_F > the switch, FP64
# after, the paper's stopping rule on the FP64 iterations
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_schedule_irsi_water100(prec):
    S, _ = config_matrix(0)
    D = blocks_to_dense(S)
    lam = float(np.linalg.eigvalsh(D)[-1])
    say(f"case schedule irsi water-100 {prec}")
    with lif.Factorization(dev(S), prec=PREC[prec], prec_switch=1e-2, start=lif.START_INV_SQRT_LMAX,
                           start_value=lam) as f:
        info = f.refine()
        Z = blocks_to_dense(f.get_Z())
        res = f.residual()
    Zm, im, _ = R.irsi(D, 32, 0.0, start="inv_sqrt_lmax", start_value=lam, prec=prec, prec_switch=1e-2)
    say(f"  gpu iterations {info['iterations_top']} reduced {info['iterations_reduced']}, oracle "
        f"{im.iterations} reduced {sum(im.reduced)}; norms {info['norms']}")
    # the switch decisions match; the last FP64 step may be a near-tie at the floor
    assert info["iterations_reduced"] == sum(im.reduced)
    assert abs(info["iterations_top"] - im.iterations) <= 1
    assert res <= 1e-12   # the FP64 floor, as the paper's rule reaches in FP64
    say(f"  rel diff vs oracle {rel(Z, Zm):.3e}")
    assert rel(Z, Zm) <= S.n * 2.0 ** -24


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_schedule_lif_chain_split_batches(prec):
    # several problems per level: in some iterations part of a level is
    # above the switch and part below, so the correction runs split
    S, cfg = config_matrix(1, count=150)   # n = 3000 chain, b = 64
    D = blocks_to_dense(S)
    tau = 1e-10
    say(f"case schedule lif chain n={S.n} {prec}")
    with lif.Factorization(dev(S), tau=tau, base_rows=512) as f:
        i64 = f.localized()
        res64 = f.residual()
    with lif.Factorization(dev(S), tau=tau, base_rows=512, prec=PREC[prec], prec_switch=1e-2) as f:
        info = f.localized()
        Z = blocks_to_dense(f.get_Z())
        res = f.residual()
    Zm, plan = R.lif(D, 64, tau, base_rows=512, prec=prec, prec_switch=1e-2)
    nodes = []

    def walk(nd):
        if nd.children:
            nodes.append(nd.info)
            walk(nd.children[0])
            walk(nd.children[1])

    walk(plan)
    red = sum(sum(i.reduced) for i in nodes)
    say(f"  gpu total {info['iterations_total']} reduced {info['iterations_reduced']} (fp64 run "
        f"{i64['iterations_total']}), oracle total {sum(i.iterations for i in nodes)} reduced {red}; "
        f"residual {res:.3e} (fp64 {res64:.3e})")
    assert info["iterations_reduced"] == red
    assert abs(info["iterations_total"] - sum(i.iterations for i in nodes)) <= len(nodes)
    assert res <= 2 * res64 + 1e-12
    say(f"  rel diff vs oracle {rel(Z, Zm):.3e}")
    assert rel(Z, Zm) <= S.n * 2.0 ** -24


# ----------------------------------------------------------------------------
# reduced delta update (update_prec): the update products with FP32 inputs in
# reduced iterations, delta formed again from its definition in FP64 when the
# schedule moves a problem to FP64.  Against the oracle's same reading: the
# switch decisions and the final factor within the FP32 accumulation bound.
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("sym", [0, 1])
def test_reduced_update_irsi_water100(prec, sym):
    S, _ = config_matrix(0)
    D = blocks_to_dense(S)
    lam = float(np.linalg.eigvalsh(D)[-1])
    say(f"case reduced update irsi water-100 {prec} sym {sym}")
    with lif.Factorization(dev(S), prec=PREC[prec], prec_switch=1e-2, start=lif.START_INV_SQRT_LMAX,
                           start_value=lam, update_prec=lif.MIXED_FP32, sym_delta=sym) as f:
        info = f.refine()
        Z = blocks_to_dense(f.get_Z())
        res = f.residual()
    Zm, im, _ = R.irsi(D, 32, 0.0, start="inv_sqrt_lmax", start_value=lam, prec=prec, prec_switch=1e-2,
                       sym_delta=bool(sym), update_prec="fp32")
    say(f"  gpu iterations {info['iterations_top']} reduced {info['iterations_reduced']}, oracle "
        f"{im.iterations} reduced {sum(im.reduced)}; norms {info['norms']} / {im.norms}")
    assert info["iterations_reduced"] == sum(im.reduced)
    assert abs(info["iterations_top"] - im.iterations) <= 1
    # the recorded norms (the one before the switch replaced by the
    # recomputed delta's) agree down to the FP64 floor, within the FP32
    # accumulation bound of the products that formed them: n 2^-24 times the
    # size of the correction, which the previous norm bounds (the last
    # reduced one is mostly that rounding: measured 5e-6 against 8e-6)
    prev = float(np.linalg.norm(np.eye(S.n) - D / lam))
    for g, o in zip(info["norms"], im.norms):
        if o > 1e-10:
            assert abs(g - o) <= 1e-6 * o + S.n * 2.0 ** -24 * prev
        prev = o
    # the refinement wins the accuracy back: the FP64 floor, tracked exactly
    assert res <= 1e-12 and abs(res - info["delta_tracked"]) <= 1e-12
    say(f"  rel diff vs oracle {rel(Z, Zm):.3e}")
    assert rel(Z, Zm) <= S.n * 2.0 ** -24


@pytest.mark.parametrize("sym", [0, 1])
def test_reduced_update_lif_chain_split_batches(sym):
    # several problems per level, split between the precisions in some
    # iterations: the update then runs in two passes
    S, cfg = config_matrix(1, count=150)   # n = 3000 chain, b = 64
    D = blocks_to_dense(S)
    tau = 1e-10
    say(f"case reduced update lif chain n={S.n} bf16 sym {sym}")
    with lif.Factorization(dev(S), tau=tau, base_rows=512, sym_delta=sym) as f:
        f.localized()
        res64 = f.residual()
    with lif.Factorization(dev(S), tau=tau, base_rows=512, prec=lif.MIXED_BF16, prec_switch=1e-2,
                           update_prec=lif.MIXED_FP32, sym_delta=sym) as f:
        info = f.localized()
        Z = blocks_to_dense(f.get_Z())
        res = f.residual()
    Zm, plan = R.lif(D, 64, tau, base_rows=512, prec="bf16", prec_switch=1e-2, sym_delta=bool(sym),
                     update_prec="fp32")
    nodes = []

    def walk(nd):
        if nd.children:
            nodes.append(nd.info)
            walk(nd.children[0])
            walk(nd.children[1])

    walk(plan)
    red = sum(sum(i.reduced) for i in nodes)
    say(f"  gpu total {info['iterations_total']} reduced {info['iterations_reduced']}, oracle total "
        f"{sum(i.iterations for i in nodes)} reduced {red}; residual {res:.3e} (fp64 {res64:.3e})")
    assert info["iterations_reduced"] == red
    assert abs(info["iterations_total"] - sum(i.iterations for i in nodes)) <= len(nodes)
    assert res <= 2 * res64 + 1e-12
    say(f"  rel diff vs oracle {rel(Z, Zm):.3e}")
    assert rel(Z, Zm) <= S.n * 2.0 ** -24


def test_reduced_update_lif_water150():
    c_, e_ = water_cluster(150, 7)
    S = overlap_blocks(c_, e_, 64)
    D = blocks_to_dense(S)
    say("case reduced update lif water-150 bf16 sym")
    with lif.Factorization(dev(S), base_rows=320, prec=lif.MIXED_BF16, prec_switch=1e-2,
                           update_prec=lif.MIXED_FP32, sym_delta=1) as f:
        info = f.localized()
        Z = blocks_to_dense(f.get_Z())
        res = f.residual()
    Zm, _ = R.lif(D, 64, 0.0, base_rows=320, prec="bf16", prec_switch=1e-2, sym_delta=True, update_prec="fp32")
    say(f"  residual {res:.3e}, reduced {info['iterations_reduced']}, rel diff vs oracle {rel(Z, Zm):.3e}")
    assert info["iterations_reduced"] > 0
    assert res <= 1e-12
    assert rel(Z, Zm) <= S.n * 2.0 ** -24
