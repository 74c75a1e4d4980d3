// Reverse sweep of refinement and localized inverse factorization for a
// linear loss L = tr(G^T Z): returns sym(dL/dS) on S's block pattern.
//
// The iteration is differentiated through the regular recurrence of
// eq. refinement_nonlocal, which produces the localized iterates in exact
// arithmetic: with delta = I - Z^T S Z and P = H_0, H_k = b_k I + delta H_{k+1},
// H_m = b_m I, one step Z' = Z P reverses to
//   Zbar_prev = Zbar' P^T,   Hbar_0 = Z^T Zbar',
//   deltabar += Hbar_k H_{k+1}^T,  Hbar_{k+1} = delta^T Hbar_k   (k < m-1),
//   deltabar += b_m Hbar_{m-1},
//   Zbar_prev -= S Z (deltabar + deltabar^T),   Sbar -= Z deltabar Z^T.
// Each checkpointed Z_i is reused as stored; delta_i and the Horner terms are
// recomputed (16 products per reversed step at m = 4).  Problems of one LIF
// level that stopped earlier pass their Zbar through unchanged.  A LIF level
// hands the diagonal parts of dL/dZ_0 = dL/d diag(Z_A, Z_C) to its children;
// the leaves (Z = U^{-1}, S = U^T U) use
//   Sbar = -Z Phi(Z^T Zbar) Z^T,  Phi = upper triangle with halved diagonal,
// which follows from Z^T dS Z = X + X^T with X = dU Z upper triangular.
// All products are FP64 and untruncated.
#include <cmath>

#include "driver.h"

namespace lif {

namespace {

std::vector<double> coeffs(int m) {
  std::vector<double> b(m + 1);
  b[0] = 1.0;
  for (int k = 1; k <= m; ++k) b[k] = b[k - 1] * (2.0 * k - 1.0) / (2.0 * k);
  return b;
}

// Reverses one level; Zbar is updated in place, Sbar accumulates.
void reverse_level(Ctx& c, const Bsr& S_full, const LevelCk& L, Bsr& Zbar, Bsr& Sbar, int m) {
  const int nn = (int)L.rlo.size();
  const int nb = S_full.nb;
  const Bsr& Sl = L.S_lvl.row_ptr.get() ? L.S_lvl : S_full;
  const std::vector<double> bk = coeffs(m);
  int kmax = 0;
  for (int k : L.iters) kmax = std::max(kmax, k);
  std::vector<int> act(nb), inact(nb);
  std::vector<unsigned char> diag(nb);
  DBuf<int> d_act(c.pool, nb), d_inact(c.pool, nb);
  DBuf<unsigned char> d_diag(c.pool, nb);
  for (int i = kmax - 1; i >= 0; --i) {
    // problems still iterating at forward step i
    std::fill(act.begin(), act.end(), -1);
    for (int s = 0; s < nn; ++s)
      if (L.iters[s] > i)
        for (int r = L.rlo[s]; r < L.rhi[s]; ++r) act[r] = s;
    for (int r = 0; r < nb; ++r) {
      inact[r] = act[r] >= 0 ? -1 : 0;
      diag[r] = act[r] >= 0 ? 1 : 0;
    }
    h2d(c, d_act.get(), act.data(), nb);
    h2d(c, d_inact.get(), inact.data(), nb);
    h2d(c, d_diag.get(), diag.data(), nb);
    Bsr Za = filter(c, L.Z[i], d_act.get(), nullptr, 2);
    Bsr Zbar_a = filter(c, Zbar, d_act.get(), nullptr, 2);
    Bsr Zbar_in = filter(c, Zbar, d_inact.get(), nullptr, 2);
    // delta_i and the Horner terms
    Bsr SZ = spgemm(c, Sl, false, Za, false, 0.0);
    Bsr ZSZ = spgemm(c, Za, true, SZ, false, 0.0);
    Bsr delta = axpby(c, -1.0, &ZSZ, 0.0, nullptr, 1.0, d_diag.get());
    ZSZ = Bsr();
    std::vector<Bsr> H(m + 1);  // H[m] = b_m I is kept implicit
    if (m >= 1) H[m - 1] = axpby(c, bk[m], &delta, 0.0, nullptr, bk[m - 1], d_diag.get());
    for (int k = m - 2; k >= 0; --k) {
      Bsr P = spgemm(c, delta, false, H[k + 1], false, 0.0);
      H[k] = axpby(c, 1.0, &P, 0.0, nullptr, bk[k], d_diag.get());
    }
    // Zbar_prev = Zbar P^T ; Hbar_0 = Z^T Zbar
    Bsr Zprev = spgemm(c, Zbar_a, false, H[0], true, 0.0);
    Bsr Hbar = spgemm(c, Za, true, Zbar_a, false, 0.0);
    Bsr dbar;
    bool have_dbar = false;
    for (int k = 0; k < m; ++k) {
      Bsr term = (k == m - 1) ? axpby(c, bk[m], &Hbar, 0.0, nullptr, 0.0, nullptr)
                              : spgemm(c, Hbar, false, H[k + 1], true, 0.0);
      dbar = have_dbar ? axpby(c, 1.0, &dbar, 1.0, &term, 0.0, nullptr) : std::move(term);
      have_dbar = true;
      if (k < m - 1) Hbar = spgemm(c, delta, true, Hbar, false, 0.0);
    }
    H.clear();
    Hbar = Bsr();
    // Zbar_prev -= S Z (dbar + dbar^T) ; Sbar -= Z dbar Z^T
    Bsr dbt = transpose(c, dbar);
    Bsr dsym = axpby(c, 1.0, &dbar, 1.0, &dbt, 0.0, nullptr);
    dbt = Bsr();
    Bsr corr = spgemm(c, SZ, false, dsym, false, 0.0);
    dsym = Bsr();
    SZ = Bsr();
    Bsr T1 = spgemm(c, Za, false, dbar, false, 0.0);
    Bsr T2 = spgemm(c, T1, false, Za, true, 0.0);
    T1 = Bsr();
    Sbar = axpby(c, 1.0, &Sbar, -1.0, &T2, 0.0, nullptr);
    Zbar = axpby3(c, 1.0, &Zbar_in, 1.0, &Zprev, -1.0, &corr);
  }
  c.sync();  // host label vectors go out of scope
}

}  // namespace

Bsr run_backward(Ctx& c, const Bsr& S, const Checkpoints& ck, const Bsr& G, const Opts& o) {
  LIF_REQUIRE(ck.valid, LIF_ERR_STATE, "no checkpoints: run lif_refine (IRSI) or lif_localized with checkpoint = 1");
  const int nb = S.nb;
  Bsr Zbar = copy(c, G);
  Bsr Sbar = bsr_empty(c, S.n, S.b);
  DBuf<int> d_part(c.pool, nb);
  for (const LevelCk& L : ck.levels) {
    reverse_level(c, S, L, Zbar, Sbar, o.m);
    if (ck.lif) {
      // dL/dZ_0 restricted to diag(Z_A, Z_C): the children's parts
      h2d(c, d_part.get(), L.part_lab.data(), nb);
      Zbar = filter(c, Zbar, d_part.get(), d_part.get(), 0);
      c.sync();
    }
  }
  if (ck.lif) {
    // leaves: Sbar -= Z Phi(Z^T Zbar) Z^T
    const Bsr& Zl = ck.Z_leaf;
    Bsr W = spgemm(c, Zl, true, Zbar, false, 0.0);
    Bsr Ph = phi_upper(c, W);
    W = Bsr();
    Bsr T = spgemm(c, Zl, false, Ph, false, 0.0);
    Bsr U = spgemm(c, T, false, Zl, true, 0.0);
    Sbar = axpby(c, 1.0, &Sbar, -1.0, &U, 0.0, nullptr);
  }
  // symmetric part on S's block pattern (zero where Sbar has no block)
  Bsr St = transpose(c, Sbar);
  Bsr sym = axpby(c, 0.5, &Sbar, 0.5, &St, 0.0, nullptr);
  St = Bsr();
  Bsr on_s = intersect(c, sym, S);
  return axpby(c, 1.0, &on_s, 0.0, &S, 0.0, nullptr);
}

}  // namespace lif
