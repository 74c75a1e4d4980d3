"""Pins of the oracle's reduced-precision delta update (the precision form
applied to the update products of eq. refinement_local, with delta formed
again from its definition when the schedule moves to FP64).

What the mathematics fixes, independently of the oracle's code:
* delta is defined as I - Z^T S Z (Sec. 2.2); while the update products run
  with FP32 inputs the tracked delta departs from that definition by FP32
  rounding (far above FP64 rounding, far below the correction itself), and
  after the move to FP64 it agrees with it to FP64 rounding again;
* the refinement wins back the accuracy of the reduced iterations: at
  tau = 0 the final factor is an inverse factor at the FP64 floor, and the
  last recorded norm is its true residual;
* with a symmetric delta the recomputed delta's blocks below the diagonal
  mirror those above bit for bit.
Planted mistakes (no recompute, an update left in FP64, a norm record not
replaced, no mirror) each fail a pin.
"""
import inspect
import textwrap

import numpy as np
import pytest

import oracle.refinement as R
from gen import blocks_to_dense, config_matrix


@pytest.fixture(scope="module")
def water100():
    S, _ = config_matrix(0)
    D = blocks_to_dense(S)
    lam = np.linalg.eigvalsh(D)
    return D, lam


def _pins(lr, D, lam, sym):
    n = D.shape[0]
    c = 1.0 / np.sqrt(lam[-1])
    I = np.eye(n)
    events = []

    def trace(k, ev, Z, d):
        events.append((k, ev, Z.copy(), d.copy()))

    Z, info = lr(D, c * I, I - c * c * D, 32, 0.0, 4, prec="bf16", prec_switch=1e-2, update_prec="fp32",
                 sym_delta=sym, trace=trace)
    ok = True
    rec = [e for e in events if e[1] == "recomputed"]
    ok &= len(rec) == 1
    if not ok:
        return False
    k_r = rec[0][0]
    for k, ev, Zk, dk in events:
        gap = np.linalg.norm(dk - (I - Zk.T @ D @ Zk))
        if ev == "updated" and info.reduced[k - 1]:
            # FP32 rounding of the update, well above FP64's
            ok &= 1e-11 < gap < 1e-4
        else:
            ok &= gap <= 1e-12
        if ev == "recomputed":
            # the norm record before iteration k_r is the recomputed delta's
            ok &= info.norms[k - 2] == float(np.sqrt(np.sum(dk * dk)))
            if sym:
                # blocks below the diagonal mirror those above bit for bit
                bi = np.arange(n) // 32
                low = bi[:, None] > bi[None, :]
                ok &= np.array_equal(dk[low], dk.T[low])
    ok &= all(info.reduced[: k_r - 1]) and not any(info.reduced[k_r - 1:])
    res = R.true_residual(D, Z)
    ok &= res <= 1e-12 and abs(res - info.norms[-1]) <= 1e-12
    return bool(ok)


@pytest.mark.parametrize("sym", [False, True])
def test_reduced_update_is_recomputed_at_the_switch(water100, sym):
    D, lam = water100
    assert _pins(R.localized_refinement, D, lam, sym)


def test_reduced_update_through_irsi_and_lif(water100):
    D, lam = water100
    Z, info, _ = R.irsi(D, 32, 0.0, start="inv_sqrt_lmax", start_value=lam[-1], prec="bf16", prec_switch=1e-2,
                        update_prec="fp32")
    assert R.true_residual(D, Z) <= 1e-12 and any(info.reduced)
    Zl, plan = R.lif(D, 32, 0.0, base_rows=128, prec="bf16", prec_switch=1e-2, update_prec="fp32")
    assert R.true_residual(D, Zl) <= 1e-12
    with pytest.raises(AssertionError):
        R.irsi(D, 32, 0.0, prec="bf16", update_prec="fp32")  # needs the schedule


def _planted(edit):
    """localized_refinement with one source edit, in the oracle's namespace."""
    src = textwrap.dedent(inspect.getsource(R.localized_refinement))
    old, new = edit
    assert src.count(old) == 1, old
    ns = dict(vars(R))
    exec(compile(src.replace(old, new), "<planted>", "exec"), ns)
    return ns["localized_refinement"]


@pytest.mark.parametrize("edit", [
    # no recompute at the switch
    ("if stale and not reduced:", "if False:"),
    # the update stays FP64 (the option ignored)
    ('pu = update_prec if reduced else "fp64"', 'pu = "fp64"'),
    # the norm record keeps the tracked value
    ("info.norms[-1] = e_cur", "pass"),
    # the recomputed delta is not mirrored
    ("                U = upper_blocks(delta, b)\n                delta = U + upper_blocks(U, b, strict=True).T\n"
     "            e_cur", "                pass\n            e_cur"),
])
def test_planted_update_prec_mistakes_are_caught(water100, edit):
    D, lam = water100
    bad = _planted(edit)
    assert not (_pins(bad, D, lam, False) and _pins(bad, D, lam, True))
