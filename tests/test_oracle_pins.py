"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each check compares the oracle with something other than itself: a closed
form (eigendecomposition, Cholesky), the spectral map of one refinement step,
the iteration bound of Sec. 3.3, the contraction bound of Sec. 2.3,
hand-derived values, a 50-digit recomputation, or finite differences.  The
planted-mistake tests at the end show that plausible slips in the oracle
(a wrong coefficient, a transposed operand, a wrong truncation comparison)
make a pin fail.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle.refinement as R
from gen import blocks_to_dense, config_matrix, dense_to_blocks, water_cluster, overlap_dense
from oracle import adjoint as ADJ
from oracle.closed_forms import (binomial_coefficients, inv_sqrt, k_max, lif_limit, predicted_norms,
                                 spectral_map, upper_inverse_factor_check)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def water100():
    S, _ = config_matrix(0)
    D = blocks_to_dense(S)
    lam = np.linalg.eigvalsh(D)
    return D, lam


def small_water(n_mol, seed=11):
    c, e = water_cluster(n_mol, seed)
    return overlap_dense(c, e)


# ----------------------------------------------------------------------------
# coefficients
# ----------------------------------------------------------------------------

def test_coefficients_match_binomial_series_and_fixture():
    got = R.coefficients(8)
    ref = binomial_coefficients(8)
    assert got == [float(x) for x in ref]
    rows = [l.split() for l in open(os.path.join(GOLDEN, "refinement_coefficients.txt")) if l[0] != "#"]
    fix = [Fraction(int(a), int(b)) for _, a, b in rows]
    assert fix == ref


def test_spectral_map_order():
    # one step maps x to f(x) with |f(x)| <= |x|^{m+1} on [-1, 1]
    x = np.linspace(-1, 1, 20001)
    for m in (1, 2, 3, 4, 6):
        f = spectral_map(x, m)
        assert np.all(np.abs(f) <= np.abs(x) ** (m + 1) + 4e-16)
    # leading term 2 b_{m+1} x^{m+1}
    x = 1e-2
    assert abs(spectral_map(x, 4) / x ** 5 - 2 * float(binomial_coefficients(5)[5])) < 1e-2


# ----------------------------------------------------------------------------
# IRSI
# ----------------------------------------------------------------------------

def test_irsi_reaches_loewdin_inverse_sqrt(water100):
    D, lam = water100
    Z, info, c = R.irsi(D, 32, 0.0, start="inv_sqrt_lmax", start_value=lam[-1])
    Zref = inv_sqrt(D)
    assert np.linalg.norm(Z - Zref) <= 1e-10 * np.linalg.norm(Zref) * 100
    assert R.true_residual(D, Z) <= 1e-12
    assert np.allclose(Z, Z.T, atol=1e-13)


def test_irsi_norms_follow_spectral_map(water100):
    D, lam = water100
    Z, info, c = R.irsi(D, 32, 0.0, start="inv_sqrt_lmax", start_value=lam[-1])
    pred = predicted_norms(1.0 - c * c * lam, 4, info.iterations)
    for got, want in zip(info.norms, pred):
        if want > 1e-9:
            assert abs(got - want) <= 1e-9 * want + 1e-12
        else:
            assert got < 1e-9
    gold = json.load(open(os.path.join(GOLDEN, "water100_oracle.json")))
    assert gold["irsi_inv_sqrt_lmax"]["iterations"] == info.iterations


def test_irsi_iteration_bound(water100):
    D, lam = water100
    # iterations to ||delta||_2 < eps never exceed K_max (eq. iter_refine_no_of_iters);
    # for Z_0 = c I with c^2 = 1/lam_max, ||delta_0||_2 = 1 - lam_min/lam_max exactly
    c = 1.0 / math.sqrt(lam[-1])
    n = D.shape[0]
    Z = c * np.eye(n)
    for eps in (1e-2, 1e-6, 1e-10):
        Zk = Z.copy()
        for k in range(1, 50):
            Zk, _ = R.nonlocal_refinement(D, Zk, 32, 0.0, iterations=1)
            d2 = np.linalg.norm(np.eye(n) - Zk.T @ D @ Zk, 2)
            if d2 < eps:
                break
        assert k <= k_max(eps, lam[0], lam[-1], 4)
    assert k_max(1e-10, lam[0], lam[-1], 4) == 6


def test_irsi_start_scales(water100):
    D, lam = water100
    beta = R.gershgorin_bound(D)
    assert beta >= lam[-1]
    for mode in ("sqrt2_over_gersh", "inv_sqrt_gersh", "optimal"):
        Z, info, c = R.irsi(D, 32, 0.0, start=mode)
        assert R.true_residual(D, Z) < 1e-11
    assert abs(R.start_scale(D, "optimal") - math.sqrt(2 / (lam[0] + lam[-1]))) < 1e-14
    assert abs(R.start_scale(D, "sqrt2_over_gersh") - math.sqrt(2 / beta)) < 1e-15


def test_two_by_two_by_hand():
    S = np.array([[1.0, 0.5], [0.5, 1.0]])
    rows = {l.split()[0]: np.array([float(v) for v in l.split()[1:]]).reshape(2, 2)
            for l in open(os.path.join(GOLDEN, "two_by_two.txt")) if l[0] != "#"}
    Z, info, c = R.irsi(S, 1, 0.0, start="optimal")
    assert np.max(np.abs(Z - rows["inv_sqrt"])) < 1e-14
    assert np.max(np.abs(R.inverse_cholesky(S) - rows["inv_chol"])) < 1e-15
    Zr = R.rinch(S, 1, 0.0, base_rows=1)
    assert np.max(np.abs(Zr - rows["inv_chol"])) < 1e-15


def test_irsi_fifty_digit_recomputation():
    # IRSI iterates recomputed in 50-digit arithmetic straight from the
    # definition delta_k = I - Z_k^T S Z_k, Z_{k+1} = Z_k sum_j b_j delta_k^j
    import mpmath as mp
    mp.mp.dps = 50
    Sf = np.array([[1.0, 0.25, 0.125, 0.0], [0.25, 1.0, 0.375, 0.0625],
                   [0.125, 0.375, 1.0, 0.5], [0.0, 0.0625, 0.5, 1.0]])
    c = 0.75
    Zf, info, _ = R.irsi(Sf, 2, 0.0, start="given", start_value=c, stop="paper")
    S = mp.matrix(Sf.tolist())
    I = mp.eye(4)
    Z = mp.mpf(c) * I
    bk = [mp.mpf(f.numerator) / f.denominator for f in binomial_coefficients(4)]
    for k in range(info.iterations):
        d = I - Z.T * S * Z
        P = bk[4] * I
        for j in (3, 2, 1, 0):
            P = bk[j] * I + d * P
        Z = Z * P
        d = I - Z.T * S * Z
        nrm = mp.sqrt(sum(d[i, j] ** 2 for i in range(4) for j in range(4)))
        if nrm > mp.mpf("1e-12"):
            assert abs(float(nrm) - info.norms[k]) <= 1e-12 * float(nrm)
    Zm = np.array([[float(Z[i, j]) for j in range(4)] for i in range(4)])
    assert np.max(np.abs(Zm - Zf)) < 1e-14


def test_identity_needs_no_iteration():
    S = np.eye(64)
    Z, info, c = R.irsi(S, 16, 0.0, start="given", start_value=1.0)
    assert info.iterations == 0 and np.array_equal(Z, np.eye(64))


def test_homogeneity_all_methods():
    D = small_water(30)
    alpha = 3.7
    Z1, _, _ = R.irsi(D, 16, 0.0, start="optimal")
    Z2, _, _ = R.irsi(alpha * D, 16, 0.0, start="optimal")
    assert np.max(np.abs(Z2 - Z1 / math.sqrt(alpha))) < 1e-12
    L1, _ = R.lif(D, 16, 0.0, base_rows=48)
    L2, _ = R.lif(alpha * D, 16, 0.0, base_rows=48)
    assert np.max(np.abs(L2 - L1 / math.sqrt(alpha))) < 1e-11
    C1 = R.rinch(D, 16, 0.0, base_rows=48)
    C2 = R.rinch(alpha * D, 16, 0.0, base_rows=48)
    assert np.max(np.abs(C2 - C1 / math.sqrt(alpha))) < 1e-11


def test_irsi_permutation_equivariant():
    D = small_water(30)
    rng = np.random.default_rng(5)
    p = rng.permutation(D.shape[0])
    Z1, _, _ = R.irsi(D, 16, 0.0)
    Z2, _, _ = R.irsi(D[np.ix_(p, p)], 16, 0.0)
    assert np.max(np.abs(Z2 - Z1[np.ix_(p, p)])) < 1e-12


def test_localized_delta_is_true_residual():
    # eq. refinement_local tracks I - Z^T S Z exactly (no truncation)
    D = small_water(30)
    n = D.shape[0]
    c = R.start_scale(D, "sqrt2_over_gersh")
    Z = c * np.eye(n)
    delta = np.eye(n) - c * c * D
    Zl, info = R.localized_refinement(D, Z, delta, 16, 0.0, m=4, stop="tol", tol=1e-6)
    Zn, _ = R.nonlocal_refinement(D, Z, 16, 0.0, m=4, iterations=info.iterations)
    assert np.max(np.abs(Zl - Zn)) < 1e-12
    assert abs(info.norms[-1] - R.true_residual(D, Zl)) < 1e-12


def test_divergent_start_is_reported():
    D = small_water(20)
    lam = np.linalg.eigvalsh(D)
    # beta = lam_max / 1.6 makes delta_0 have eigenvalues below -1
    with pytest.raises(R.NoConvergence):
        R.irsi(D, 16, 0.0, start="given", start_value=math.sqrt(1.6 / lam[-1]) * math.sqrt(1.6))


def test_not_positive_definite():
    D = small_water(10)
    D[3, 3] = -1.0
    with pytest.raises(R.NotPositiveDefinite):
        R.lif(D, 16, 0.0, base_rows=32)


# ----------------------------------------------------------------------------
# RINCH and LIF
# ----------------------------------------------------------------------------

def test_rinch_is_inverse_cholesky(water100):
    D, _ = water100
    Z = R.rinch(D, 32, 0.0, base_rows=128)
    low, dmin, res = upper_inverse_factor_check(D, Z)
    assert low == 0.0 and dmin > 0 and res < 1e-12
    Zf = R.inverse_cholesky(D)
    low, dmin, res = upper_inverse_factor_check(D, Zf)
    assert low == 0.0 and dmin > 0 and res < 1e-12
    assert np.max(np.abs(Z - Zf)) < 1e-12 * np.max(np.abs(Zf))


def test_lif_reaches_recursive_limit(water100):
    D, _ = water100
    Z, plan = R.lif(D, 32, 0.0, base_rows=128)
    Zref = lif_limit(D, 32, 128)
    assert np.linalg.norm(Z - Zref) <= 1e-13 * np.linalg.norm(Zref) * 10
    assert R.true_residual(D, Z) < 1e-12


def test_lif_contraction_bound_and_norms(water100):
    D, _ = water100
    Z, plan = R.lif(D, 32, 0.0, base_rows=128)

    def walk(node):
        if not node.children:
            return
        Sn = D[node.lo:node.hi, node.lo:node.hi]
        lam = np.linalg.eigvalsh(Sn)
        # Sec. 2.3: ||I - Z_0^T S Z_0||_2 <= 1 - lam_min / lam_max
        assert node.delta0_norm2 <= 1 - lam[0] / lam[-1] + 1e-12
        # the node's norms follow the spectral map from delta_0's eigenvalues
        a, c = node.children
        Z0 = np.zeros_like(Sn)
        h = a.hi - a.lo
        Z0[:h, :h] = lif_limit(Sn[:h, :h], 32, 128)
        Z0[h:, h:] = lif_limit(Sn[h:, h:], 32, 128)
        mu = np.linalg.eigvalsh(np.eye(Sn.shape[0]) - Z0.T @ Sn @ Z0)
        pred = predicted_norms(mu, 4, node.info.iterations)
        for got, want in zip(node.info.norms, pred):
            if want > 1e-8:
                assert abs(got - want) <= 1e-8 * want
        walk(a)
        walk(c)

    walk(plan)
    assert plan.children and plan.info.iterations >= 2


def test_nonlocal_irsi_reaches_loewdin_and_spectral_map(water100):
    # the regular form from Z_0 = c I: same limit (S^{-1/2}) and, in exact
    # arithmetic, the same norms as the localized form (spectral map of delta_0)
    D, lam = water100
    Z, info, c = R.irsi(D, 32, 0.0, start="inv_sqrt_lmax", start_value=lam[-1], refinement="nonlocal")
    Zref = inv_sqrt(D)
    assert np.linalg.norm(Z - Zref) <= 1e-10 * np.linalg.norm(Zref) * 100
    assert R.true_residual(D, Z) <= 1e-12
    pred = predicted_norms(1.0 - c * c * lam, 4, info.iterations)
    for got, want in zip(info.norms, pred):
        if want > 1e-9:
            assert abs(got - want) <= 1e-9 * want + 1e-12
    Zl, infol, _ = R.irsi(D, 32, 0.0, start="inv_sqrt_lmax", start_value=lam[-1])
    assert info.iterations == infol.iterations


def test_nonlocal_lif_reaches_recursive_limit(water100):
    # recursive inverse factorization with the regular correction (Sec. 2.3)
    # has the limit of LIF: each node's refinement converges to
    # Z_0 (Z_0^T S_n Z_0)^{-1/2} from the same Z_0, with delta_0 = I - Z_0^T S Z_0
    D, _ = water100
    Z, plan = R.lif(D, 32, 0.0, base_rows=128, refinement="nonlocal")
    Zref = lif_limit(D, 32, 128)
    assert np.linalg.norm(Z - Zref) <= 1e-13 * np.linalg.norm(Zref) * 10
    assert R.true_residual(D, Z) < 1e-12

    def walk(node):
        if not node.children:
            return
        Sn = D[node.lo:node.hi, node.lo:node.hi]
        a, c = node.children
        Z0 = np.zeros_like(Sn)
        h = a.hi - a.lo
        Z0[:h, :h] = lif_limit(Sn[:h, :h], 32, 128)
        Z0[h:, h:] = lif_limit(Sn[h:, h:], 32, 128)
        mu = np.linalg.eigvalsh(np.eye(Sn.shape[0]) - Z0.T @ Sn @ Z0)
        pred = predicted_norms(mu, 4, node.info.iterations)
        for got, want in zip(node.info.norms, pred):
            if want > 1e-8:
                assert abs(got - want) <= 1e-8 * want
        walk(a)
        walk(c)

    walk(plan)
    assert plan.children and plan.info.iterations >= 2
    _, plan_l = R.lif(D, 32, 0.0, base_rows=128)
    assert plan.info.iterations == plan_l.info.iterations


def test_lif_block_diagonal_needs_no_iteration():
    D = small_water(12)
    n = D.shape[0]
    h = R.split_point(n, 16)
    D[:h, h:] = 0.0
    D[h:, :h] = 0.0
    Z, plan = R.lif(D, 16, 0.0, base_rows=n - 1)
    assert plan.info.iterations == 0
    assert np.array_equal(Z[:h, h:], np.zeros((h, n - h)))


def test_lif_plan_split_rule():
    plan = R.lif_plan(100_000, 64, 4096)
    leaves = []

    def walk(nd):
        if nd.children:
            a, c = nd.children
            assert a.lo % 64 == 0 and c.lo % 64 == 0 and a.hi == c.lo
            nb = (nd.hi - nd.lo + 63) // 64
            assert (a.hi - a.lo) == ((nb + 1) // 2) * 64
            walk(a)
            walk(c)
        else:
            leaves.append(nd)

    walk(plan)
    assert len(leaves) == 32 and all(l.hi - l.lo <= 4096 for l in leaves) and leaves[-1].hi == 100_000
    assert {l.depth for l in leaves} == {5}


# ----------------------------------------------------------------------------
# truncation
# ----------------------------------------------------------------------------

def test_truncation_threshold_is_strict():
    b = 4
    X = np.zeros((8, 8))
    X[0:4, 4:8] = 0.25            # norm exactly 1.0 -> kept at tau = 1
    X[4:8, 0:4] = 0.25 * (1 - 1e-12)  # just below -> dropped
    X[4:8, 4:8] = 2.0
    T = R.truncate(X, b, 1.0)
    assert np.array_equal(T[0:4, 4:8], X[0:4, 4:8])
    assert not np.any(T[4:8, 0:4])
    assert np.array_equal(T[4:8, 4:8], X[4:8, 4:8])
    assert np.array_equal(R.truncate(X, b, 0.0), X)


def test_truncated_methods_order_and_floor(water100):
    # Sec. 5.4 (Table 1): RINCH most accurate, IRSI least, LIF in between (tau > 0)
    D, _ = water100
    tau = 1e-5
    Dt = R.truncate(D, 32, tau)
    Zi, _, _ = R.irsi(D, 32, tau)
    Zl, _ = R.lif(D, 32, tau, base_rows=128)
    Zr = R.rinch(D, 32, tau, base_rows=128)
    ei, el, er = (R.true_residual(Dt, z) for z in (Zi, Zl, Zr))
    assert er < el < ei
    assert ei < 1e3 * tau


# ----------------------------------------------------------------------------
# adjoints against finite differences and eigendecomposition references
# ----------------------------------------------------------------------------

def _spd(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    return A @ A.T / n + np.eye(n), rng


def _fd(fun, S, E, h=1e-6):
    return (fun(S + h * E) - fun(S - h * E)) / (2 * h)


def test_inverse_cholesky_grad_fd():
    S, rng = _spd(40, 1)
    G = rng.standard_normal(S.shape)
    E = rng.standard_normal(S.shape)
    E = E + E.T
    g = np.sum(ADJ.inverse_cholesky_grad(S, G) * E)
    fd = _fd(lambda s: np.sum(G * R.inverse_cholesky(s)), S, E)
    assert abs(g - fd) <= 1e-7 * abs(fd)


def test_irsi_grad_fd_and_eigen_reference():
    S, rng = _spd(40, 2)
    G = rng.standard_normal(S.shape)
    E = rng.standard_normal(S.shape)
    E = E + E.T
    lam = np.linalg.eigvalsh(S)
    c = 1 / math.sqrt(lam[-1])
    K = 8
    g = np.sum(ADJ.irsi_grad(S, G, c, 4, K) * E)
    fd = _fd(lambda s: np.sum(G * ADJ.refine_forward(s, c * np.eye(40), 4, K)[-1]), S, E)
    assert abs(g - fd) <= 1e-7 * abs(fd)
    ref = np.sum(ADJ.inv_sqrt_grad(S, G) * E)
    assert abs(g - ref) <= 1e-9 * abs(ref)
    fd2 = _fd(lambda s: np.sum(G * inv_sqrt(s)), S, E)
    assert abs(ref - fd2) <= 1e-7 * abs(fd2)


def test_lif_grad_fd_and_limit_reference():
    S, rng = _spd(60, 3)
    G = rng.standard_normal(S.shape)
    E = rng.standard_normal(S.shape)
    E = E + E.T
    iters = {}

    def collect(lo, hi):
        if hi - lo <= 16:
            return
        h = R.split_point(hi - lo, 8)
        iters[(lo, hi)] = 7
        collect(lo, lo + h)
        collect(lo + h, hi)

    collect(0, 60)
    g = np.sum(ADJ.lif_grad(S, G, 8, 16, 4, iters) * E)
    fd = _fd(lambda s: np.sum(G * ADJ.lif_forward_regular(s, 8, 16, 4, iters)[0]), S, E)
    assert abs(g - fd) <= 1e-7 * abs(fd)
    ref = np.sum(ADJ.lif_limit_grad(S, G, 8, 16) * E)
    assert abs(g - ref) <= 1e-9 * abs(ref)
    fd2 = _fd(lambda s: np.sum(G * lif_limit(s, 8, 16)), S, E)
    assert abs(ref - fd2) <= 1e-7 * abs(fd2)


# ----------------------------------------------------------------------------
# planted mistakes: each must make a pin above fail
# ----------------------------------------------------------------------------

def test_planted_wrong_coefficient_is_caught(monkeypatch, water100):
    good = R.coefficients

    def bad(m):
        b = good(m)
        b[3] *= 1.01
        return b

    monkeypatch.setattr(R, "coefficients", bad)
    with pytest.raises(AssertionError):
        test_irsi_norms_follow_spectral_map(water100)


def test_planted_transposed_leaf_is_caught(monkeypatch, water100):
    good = R.inverse_cholesky
    monkeypatch.setattr(R, "inverse_cholesky", lambda S: good(S).T)
    with pytest.raises((AssertionError, R.NotPositiveDefinite)):
        test_rinch_is_inverse_cholesky(water100)


def test_planted_delta_sign_is_caught(monkeypatch):
    # delta_0 built with the wrong sign must break the LIF limit pin
    good = R.localized_refinement

    def bad(S, Z0, delta0, *a, **k):
        return good(S, Z0, -delta0, *a, **k)

    monkeypatch.setattr(R, "localized_refinement", bad)
    D = small_water(40)
    with pytest.raises((AssertionError, R.NoConvergence)):
        Z, _ = R.lif(D, 16, 0.0, base_rows=96)
        assert np.linalg.norm(Z - lif_limit(D, 16, 96)) <= 1e-10 * np.linalg.norm(Z)


def test_planted_truncation_comparison_is_caught(monkeypatch):
    monkeypatch.setattr(R, "truncate", lambda X, b, tau: X if tau <= 0 else np.where(
        np.repeat(np.repeat(R.block_norms(X, b) > tau, b, 0), b, 1)[:X.shape[0], :X.shape[1]], X, 0.0))
    with pytest.raises(AssertionError):
        test_truncation_threshold_is_strict()


# ----------------------------------------------------------------------------
# precision form: input rounding
# ----------------------------------------------------------------------------

def test_bf16_and_fp32_rounding_by_hand():
    # BF16 keeps 8 significant bits (7 stored); ties go to the even pattern
    one = 1.0
    cases = [
        (1.0 + 2.0 ** -8, 1.0),                   # exact tie, 1.0 is even
        (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),   # tie between 1+2^-7 (odd) and 1+2^-6 (even)
        (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),  # just above the tie
        (-(1.0 + 2.0 ** -8), -1.0),
        (3.0, 3.0), (0.0, 0.0),
        (2.0 ** -130, 2.0 ** -130),               # FP32 subnormal, representable in BF16
    ]
    got = R.round_to(np.array([c[0] for c in cases]), "bf16")
    assert np.array_equal(got, np.array([c[1] for c in cases]))
    assert np.isinf(R.round_to(np.array([np.inf]), "bf16"))[0]
    assert np.isnan(R.round_to(np.array([np.nan]), "bf16"))[0]
    # FP32: 24 significant bits
    x = np.array([1.0 + 2.0 ** -24, 1.0 + 3 * 2.0 ** -24, 0.1])
    assert np.array_equal(R.round_to(x, "fp32"), np.array([1.0, 1.0 + 2.0 ** -22, float(np.float32(0.1))]))
    assert R.round_to(np.array([one]), "fp64")[0] == one


def _mult_add_pins(fn):
    """The precision form's reading of a Horner step delta (X + c I): only
    delta and X are rounded, c delta enters in FP64, alpha scales the
    product of the rounded inputs."""
    rng = np.random.Generator(np.random.PCG64(3))
    n, b = 40, 8
    d = rng.standard_normal((n, n))
    ok = True
    # X = 0: the product vanishes and the result is c delta exactly (not c round(delta))
    c = 0.3125
    got = fn(d, np.zeros((n, n)), b, 0.0, "bf16", D=d, gamma=c)
    ok &= bool(np.array_equal(got, c * d))
    # entries 1 + 2^-7 are BF16 numbers; b_4 = 35/128 times their square sum is
    # exact in FP64 but b_4 (1 + 2^-7) is not a BF16 number: the scaling must
    # act on the product of the rounded inputs, not on an input
    e = np.full((n, n), 1.0 + 2.0 ** -7)
    a4 = 35.0 / 128.0
    want = a4 * n * (1.0 + 2.0 ** -7) ** 2 * np.ones((n, n))
    ok &= bool(np.array_equal(fn(e, e, b, 0.0, "bf16", alpha=a4), want))
    # FP64: the fused form equals the product with the explicit factor X + c I
    X = rng.standard_normal((n, n))
    ref = d @ (X + c * np.eye(n))
    ok &= bool(np.max(np.abs(fn(d, X, b, 0.0, "fp64", D=d, gamma=c) - ref)) <= 1e-13 * np.max(np.abs(ref)))
    # bf16: within the input rounding of delta and X of the exact value
    u = 2.0 ** -8
    err = np.abs(fn(d, X, b, 0.0, "bf16", D=d, gamma=c) - ref)
    ok &= bool(np.all(err <= 2.01 * u * (np.abs(d) @ np.abs(X)) + 1e-15 * np.abs(ref)))
    return ok


def test_mult_add_reading_of_the_horner_step():
    assert _mult_add_pins(R.mult_add)


def test_planted_rounded_identity_term_is_caught():
    def bad(A, B, b, tau, prec="fp64", alpha=1.0, D=None, gamma=0.0):
        # rounds the whole factor T = X + c I (D = A here)
        T = alpha * B + gamma * np.eye(B.shape[0])
        return R.truncate(R.round_to(A, prec) @ R.round_to(T, prec), b, tau)

    def bad_alpha(A, B, b, tau, prec="fp64", alpha=1.0, D=None, gamma=0.0):
        P = R.round_to(alpha * A, prec) @ R.round_to(B, prec)
        if D is not None and gamma != 0.0:
            P = P + gamma * D
        return R.truncate(P, b, tau)
    assert not _mult_add_pins(bad)
    assert not _mult_add_pins(bad_alpha)


def test_precision_schedule_reaches_fp64_floor(water100):
    # precision schedule: reduced-precision corrections while ||delta||_F
    # exceeds the switch, FP64 after, the paper's rule on the FP64 iterations.
    # The result is an inverse factor at the FP64 floor, the reduced
    # iterations are exactly those that start above the switch, and the
    # count stays within one of the FP64 run's.
    D, lam = water100
    n = D.shape[0]
    Z64, i64, c = R.irsi(D, 32, 0.0, start="inv_sqrt_lmax", start_value=lam[-1])
    e0 = float(np.linalg.norm(np.eye(n) - c * c * D))
    for prec, u_in in (("fp32", 2.0 ** -24), ("bf16", 2.0 ** -8)):
        Z, info, _ = R.irsi(D, 32, 0.0, start="inv_sqrt_lmax", start_value=lam[-1], prec=prec, prec_switch=1e-2)
        res = R.true_residual(D, Z)
        assert res <= 1e-12 and abs(res - info.norms[-1]) <= 1e-12
        before = [e0] + info.norms[:-1]
        assert info.reduced == [e > 1e-2 for e in before]
        assert any(info.reduced) and not all(info.reduced)
        assert info.iterations <= i64.iterations + 1
        dev = np.linalg.norm(Z - Z64) / np.linalg.norm(Z64)
        assert dev <= 10 * u_in
    # per LIF node as well
    _, plan64 = R.lif(D, 32, 0.0, base_rows=128)
    Z, plan = R.lif(D, 32, 0.0, base_rows=128, prec="bf16", prec_switch=1e-2)
    assert R.true_residual(D, Z) <= 1e-12
    assert any(plan.info.reduced) and not plan.info.reduced[-1]
    assert plan.info.iterations <= plan64.info.iterations + 1


def test_symmetric_delta_reaches_closed_forms(water100):
    # delta is symmetric in exact arithmetic: updating its upper block
    # triangle and mirroring it keeps the limits and the spectral-map norms
    D, lam = water100
    Z, info, c = R.irsi(D, 32, 0.0, start="inv_sqrt_lmax", start_value=lam[-1], sym_delta=True)
    Zref = inv_sqrt(D)
    assert np.linalg.norm(Z - Zref) <= 1e-10 * np.linalg.norm(Zref) * 100
    assert R.true_residual(D, Z) <= 1e-12
    pred = predicted_norms(1.0 - c * c * lam, 4, info.iterations)
    for got, want in zip(info.norms, pred):
        if want > 1e-9:
            assert abs(got - want) <= 1e-9 * want + 1e-12
    Zl, plan = R.lif(D, 32, 0.0, base_rows=128, sym_delta=True)
    assert np.linalg.norm(Zl - lif_limit(D, 32, 128)) <= 1e-12 * np.linalg.norm(Zl)
    # the mirror: a matrix with a ragged last block, upper part kept, lower rebuilt
    A = np.arange(49.0).reshape(7, 7)
    U = R.upper_blocks(A, 3)
    assert U[4, 1] == 0.0 and U[1, 4] == A[1, 4] and U[4, 4] == A[4, 4] and U[5, 6] == A[5, 6] and U[6, 5] == 0.0
    assert R.upper_blocks(A, 3, strict=True)[4, 4] == 0.0


def test_mixed_refinement_reaches_fp64_accuracy(water100):
    # the refinement wins back the accuracy lost in the correction products:
    # with FP64 delta updates the tracked delta is the true residual, and TOL
    # stopping reaches 1e-10 for FP32 and BF16 inputs.  The factor reached is
    # an inverse factor (Z^T S Z = I) within O(u_in) of the FP64 one, u_in the
    # unit roundoff of the inputs: inexact corrections move Z along the set of
    # inverse factors, which the residual does not see.
    D, lam = water100
    Z64, i64, _ = R.irsi(D, 32, 0.0, start="inv_sqrt_lmax", start_value=lam[-1], stop="tol", tol=1e-10)
    for prec, u_in in (("fp32", 2.0 ** -24), ("bf16", 2.0 ** -8)):
        Z, info, _ = R.irsi(D, 32, 0.0, start="inv_sqrt_lmax", start_value=lam[-1], stop="tol", tol=1e-10,
                            prec=prec)
        assert info.norms[-1] <= 1e-10 and not info.stagnated
        assert abs(R.true_residual(D, Z) - info.norms[-1]) <= 1e-12
        assert info.iterations >= i64.iterations
        dev = np.linalg.norm(Z - Z64) / np.linalg.norm(Z64)
        assert 0.01 * u_in < dev <= 10 * u_in
