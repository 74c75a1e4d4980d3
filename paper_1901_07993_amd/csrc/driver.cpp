// Refinement and localized-recursion drivers (host code).
#include "driver.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>

namespace lif {

namespace {

// Coefficients of eq. refinement_nonlocal: b_0 = 1, b_k = (2k-1)/(2k) b_{k-1}.
std::vector<double> coefficients(int m) {
  std::vector<double> b(m + 1);
  b[0] = 1.0;
  for (int k = 1; k <= m; ++k) b[k] = b[k - 1] * (2.0 * k - 1.0) / (2.0 * k);
  return b;
}

// Stopping decision after delta_k of one problem has been formed.
//   paper rule (Sec. 2.2): stop when e_k > e_{k-1}^{m+1}; the error record
//     starts at the largest real value and its (m+1)-th power, so the first
//     real comparison is k = 2; delta_k = 0 also stops.
//   tol rule: stop when e_k <= tol or when e_k >= e_{k-1} (no progress).
// A norm that grows while >= 1 is divergence (the start was not a
// contraction); a non-finite norm likewise.
enum class Step { Continue, Stop, Diverged };

// `test` false (an iteration with a reduced-precision correction under the
// precision schedule, which converges linearly): divergence checks only.
Step stop_decision(int k, double e, double e_prev, bool has_prev, int m, int stop, double tol, bool* stagnated,
                   bool test) {
  if (!std::isfinite(e)) return Step::Diverged;
  if (has_prev && e > e_prev && e >= 1.0) return Step::Diverged;
  if (!test) return Step::Continue;
  if (stop == LIF_STOP_PAPER) {
    if (e == 0.0) return Step::Stop;
    if (has_prev && e > std::pow(e_prev, m + 1)) return Step::Stop;
    return Step::Continue;
  }
  if (e <= tol) return Step::Stop;
  if (has_prev && e >= e_prev) {
    *stagnated = true;
    return Step::Stop;
  }
  return Step::Continue;
}

// An iteration whose products (with margins) would take more than this is
// not sized in advance.
constexpr double kPlanIterBytes = 4.0 * double(1u << 30);
// Capacities carried over from the level below predict the next level's
// first iteration only roughly (its problems are twice as large); they are
// used while they describe small products, where a read-back would cost more
// than the rare redone iteration.
constexpr double kPlanCarryBytes = 256.0 * double(1u << 20);

struct NodeState {
  bool active = true;
  bool has_prev = false;
  double e_prev = 0.0;
  double e = 0.0;
  double e_cur = 0.0;   // ||delta||_F before the next iteration
  int iterations = 0;
  int reduced = 0;      // iterations whose correction ran in reduced precision
  bool stagnated = false;
  std::vector<double> norms;
};

// A set of independent problems refined together: node s owns block rows
// [rlo[s], rhi[s]).  S is the matching block-diagonal part of the matrix.
struct Batch {
  std::vector<int> rlo, rhi;
  int nb = 0;
};

// delta = I - trunc(trunc(Z^T S) Z) on the block rows flagged in `on`, the
// residual of the regular form (eq. refinement_nonlocal).  Both products
// keep their dropped blocks as holes: only the sum reads them.
Bsr regular_delta(Ctx& c, const Bsr& S, const Bsr& Z, double tau, const unsigned char* on) {
  Bsr W = spgemm(c, Z, true, S, false, tau, LIF_FP64, 1.0, nullptr, 0.0, true);
  Bsr V = spgemm(c, W, false, Z, false, tau, LIF_FP64, 1.0, nullptr, 0.0, true);
  W = Bsr();
  return axpby(c, -1.0, &V, 0.0, nullptr, 1.0, on);
}

// `carry` (nullable): product capacities handed from one batch to the next
// of the same factorization; the first iteration is then sized in advance
// too (and redone with exact sizes if a capacity was short).
// `ss0` (nullable): the problems' ||delta_0||_F^2, when the caller already
// read them back.
void refine_batch(Ctx& c, const Bsr& S, Bsr& Z, Bsr delta, const Batch& bt, const Opts& o,
                  std::vector<NodeState>& st, int max_iter, std::vector<Bsr>* ck = nullptr,
                  std::vector<std::array<int64_t, 2>>* carry = nullptr, const std::vector<double>* ss0 = nullptr) {
  const int nn = (int)bt.rlo.size();
  const int nb = bt.nb;
  const std::vector<double> bk = coefficients(o.m);
  st.assign(nn, NodeState());
  DBuf<int> d_rlo(c.pool, nn), d_rhi(c.pool, nn);
  h2d(c, d_rlo.get(), bt.rlo.data(), nn);
  h2d(c, d_rhi.get(), bt.rhi.data(), nn);

  {  // problems whose delta_0 is exactly zero need no iteration
    const std::vector<double> ss = ss0 ? *ss0 : node_sumsq(c, delta, d_rlo.get(), d_rhi.get(), nn);
    for (int s = 0; s < nn; ++s) {
      st[s].e_cur = std::sqrt(ss[s]);
      if (ss[s] == 0.0) st[s].active = false;
    }
  }

  std::vector<int> rowlab(nb);
  DBuf<int> d_rowlab(c.pool, nb);
  // regular form: the identity of delta = I - Z^T S Z lives on the rows of
  // the batch's problems only
  const bool regular = o.refinement == LIF_REFINE_NONLOCAL;
  DBuf<unsigned char> d_inb;
  std::vector<unsigned char> inb;  // host source of an async copy: lives to the end
  Bsr none;
  if (regular) {
    inb.assign(nb, 0);
    for (int s = 0; s < nn; ++s)
      for (int i = bt.rlo[s]; i < bt.rhi[s]; ++i) inb[i] = 1;
    d_inb = DBuf<unsigned char>(c.pool, nb);
    h2d(c, d_inb.get(), inb.data(), nb);
    none = bsr_empty(c, S.n, S.b);
  }
  bool labels_dirty = true;
  bool all_active = true;
  std::vector<std::array<int64_t, 2>> caps;  // per product of an iteration: {blocks, pairs}
  if (carry) caps = *carry;
  // Under the precision schedule the problems of a batch may need different
  // precisions in one iteration; the correction products then run twice, on
  // each group's rows (the sequence of products, and so the capacities of an
  // iteration, differs: caps_split records which sequence caps describes).
  bool caps_split = false;
  std::vector<char> red(nn, 0);
  std::vector<int> lab_red(nb), lab_full(nb);
  DBuf<int> d_lab_red, d_lab_full;
  // symmetric delta: block-index labels (i and i + 1) select the upper and
  // the strictly upper block triangles
  std::vector<int> iota, iota1;
  DBuf<int> d_iota, d_iota1;
  if (o.sym_delta) {
    iota.resize(nb);
    iota1.resize(nb);
    for (int i = 0; i < nb; ++i) {
      iota[i] = i;
      iota1[i] = i + 1;
    }
    d_iota = DBuf<int>(c.pool, nb);
    d_iota1 = DBuf<int>(c.pool, nb);
    h2d(c, d_iota.get(), iota.data(), nb);
    h2d(c, d_iota1.get(), iota1.data(), nb);
  }
  // delta_{k+1} from delta_k and the two products: the full difference, or
  // with a symmetric delta the difference on the upper block triangle (the
  // products hold only those blocks) with its strictly upper part mirrored
  // the upper block triangle of U with its strictly upper part mirrored below
  auto mirror_upper = [&](const Bsr& U) {
    Bsr L;
    {
      Bsr SU = filter(c, U, d_iota1.get(), d_iota.get(), 3);
      L = transpose(c, SU);
    }
    return axpby(c, 1.0, &U, 1.0, &L, 0.0, nullptr);
  };
  auto delta_update_from = [&](const Bsr& d0, const Bsr& X1, const Bsr& X2) {
    if (!o.sym_delta) return axpby3(c, 1.0, &d0, -1.0, &X1, -1.0, &X2);
    Bsr U;
    {
      Bsr dU = filter(c, d0, d_iota.get(), d_iota.get(), 3);
      U = axpby3(c, 1.0, &dU, -1.0, &X1, -1.0, &X2);
    }
    return mirror_upper(U);
  };
  auto delta_update = [&](const Bsr& X1, const Bsr& X2) { return delta_update_from(delta, X1, X2); };
  // The update on large problems, formed by panels of block rows so that
  // neither product is ever held whole: rows [p0, p1) of Z_{k+1}^T (S M) take
  // Z_{k+1}'s block columns in [p0, p1), rows of (S M)^T Z_k the same columns
  // of S M; each output block is the whole product's block (same block
  // products in the same order), so the result is bit for bit that of the
  // whole update.  The panels' row sets are disjoint: joining them moves
  // pointers only, and like the assembly of submatrices it is not a task.
  DBuf<int> d_pzero, d_plab, d_piota;
  auto delta_update_panels = [&](const Bsr& d0, const Bsr& SM, const Bsr& Zk, const Bsr& Zn, int rows, int pu) {
    if (!d_pzero.get()) {
      d_pzero = DBuf<int>(c.pool, nb);
      d_plab = DBuf<int>(c.pool, nb);
      launch_fill_i32(c, d_pzero.get(), 0, nb);
      if (o.sym_delta) d_piota = DBuf<int>(c.pool, nb);
    }
    Bsr acc;
    bool have = false;
    int part_cpl = 0, part_prod = 0;
    for (int p0 = 0; p0 < nb; p0 += rows) {
      const int p1 = std::min(nb, p0 + rows);
      // label 0 on the panel's block indices, -1 elsewhere
      launch_fill_i32(c, d_plab.get(), -1, nb);
      launch_fill_i32(c, d_plab.get() + p0, 0, p1 - p0);
      Bsr X1, X2;
      {
        Bsr Zc = filter(c, Zn, d_pzero.get(), d_plab.get(), 0);
        X1 = spgemm(c, Zc, true, SM, false, o.tau, pu, 1.0, nullptr, 0.0, true, false, o.sym_delta);
      }
      {
        Bsr Sc = filter(c, SM, d_pzero.get(), d_plab.get(), 0);
        X2 = spgemm(c, Sc, true, Zk, false, o.tau, pu, 1.0, nullptr, 0.0, true, false, o.sym_delta);
      }
      Bsr dP;
      if (o.sym_delta) {
        // the panel's rows of delta's upper block triangle
        launch_fill_i32(c, d_piota.get(), -1, nb);
        LIF_HIP(hipMemcpyAsync(d_piota.get() + p0, d_iota.get() + p0, (size_t)(p1 - p0) * sizeof(int),
                               hipMemcpyDeviceToDevice, c.stream));
        dP = filter(c, d0, d_piota.get(), d_iota.get(), 3);
      } else {
        dP = filter(c, d0, d_plab.get(), nullptr, 2);
      }
      Bsr part = axpby3(c, 1.0, &dP, -1.0, &X1, -1.0, &X2);
      if (part.cpl > part_cpl || (part.cpl == part_cpl && part.cpl_products > part_prod)) {
        part_cpl = part.cpl;
        part_prod = part.cpl_products;
      }
      if (!have) {
        acc = std::move(part);
        have = true;
      } else {
        const int sc = c.stats.cpl, sp = c.stats.cpl_products;
        acc = axpby(c, 1.0, &acc, 1.0, &part, 0.0, nullptr);
        c.stats.cpl = sc;
        c.stats.cpl_products = sp;
      }
    }
    acc.cpl = part_cpl;
    acc.cpl_products = part_prod;
    if (!o.sym_delta) return acc;
    return mirror_upper(acc);
  };
  const bool up = o.sym_delta;
  // The input-precision copies the update's products made of Z_k and Z_{k+1}
  // (transposed operands) have no other reader: on one stream their memory
  // is given back as soon as the products are queued.
  auto drop_update_copies = [&](const Bsr& Zk, const Bsr& Zn, int pu) {
    if (pu == LIF_FP64) return;
    Zk.lp[1] = Bsr::Shadow();
    Zn.lp[1] = Bsr::Shadow();
  };
  // d0 - Z_{k+1}^T (S Mp) - (S Mp)^T Z_k with the products in precision pu,
  // on one stream, by panels when large (the correction Mp may be that of
  // some of the problems only: the others' rows of d0 pass unchanged)
  auto update_pass = [&](const Bsr& d0, const Bsr& Mp, const Bsr& Zk, const Bsr& Zn, bool planned_it, int pu) {
    const bool lp = pu != LIF_FP64;  // S M's input-precision copy, read by both products
    Bsr SM = spgemm(c, S, false, Mp, false, o.tau, pu, 1.0, nullptr, 0.0, true, lp);
    int prow = o.update_panel_rows;
    if (prow == 0 && !planned_it) {
      const double upd = (o.sym_delta ? 1.0 : 2.0) * (double)d0.bound() * S.b * S.b * sizeof(double);
      const double dev = (double)c.device_bytes();
      if (upd > dev / 16.0) {
        const int np = (int)std::ceil(upd / (dev / 32.0));
        prow = (nb + np - 1) / np;
      }
    }
    Bsr d1;
    if (prow > 0 && prow < nb) {
      d1 = delta_update_panels(d0, SM, Zk, Zn, prow, pu);
    } else {
      Bsr X2 = spgemm(c, SM, true, Zk, false, o.tau, pu, 1.0, nullptr, 0.0, true, false, up);
      Bsr X1 = spgemm(c, Zn, true, SM, false, o.tau, pu, 1.0, nullptr, 0.0, true, false, up);
      SM = Bsr();
      d1 = delta_update_from(d0, X1, X2);
    }
    drop_update_copies(Zk, Zn, pu);
    return d1;
  };
  // Reduced delta update (update_prec): per problem, whether its delta
  // carries the rounding of reduced-precision updates.  When the schedule
  // moves a problem to FP64, its delta is formed again from the definition,
  // I - trunc(Z^T trunc(S Z)) (Sec. 2.2; S Z first, as the update forms S M,
  // and with a symmetric delta only the upper block triangle of the second
  // product; the problems share no block, so this runs on their rows of Z),
  // and its norm replaces the last recorded one.
  const bool red_update = o.update_prec != LIF_FP64 && o.prec != LIF_FP64 && !regular;
  std::vector<char> stale(nn, 0);
  std::vector<int> lab_sw(nb), lab_keep(nb);  // host sources of async copies: live to the end
  std::vector<unsigned char> on_sw(nb);
  DBuf<int> d_lab_sw, d_lab_keep;
  DBuf<unsigned char> d_on_sw;
  auto recompute_delta = [&](const std::vector<char>& sw) {
    for (int i = 0; i < nb; ++i) {
      lab_sw[i] = lab_keep[i] = -1;
      on_sw[i] = 0;
    }
    for (int s = 0; s < nn; ++s)
      for (int i = bt.rlo[s]; i < bt.rhi[s]; ++i) {
        (sw[s] ? lab_sw : lab_keep)[i] = s;
        on_sw[i] = sw[s] ? 1 : 0;
      }
    if (!d_lab_sw.get()) {
      d_lab_sw = DBuf<int>(c.pool, nb);
      d_lab_keep = DBuf<int>(c.pool, nb);
      d_on_sw = DBuf<unsigned char>(c.pool, nb);
    }
    h2d(c, d_lab_sw.get(), lab_sw.data(), nb);
    h2d(c, d_lab_keep.get(), lab_keep.data(), nb);
    h2d(c, d_on_sw.get(), on_sw.data(), nb);
    Bsr dn;
    {
      Bsr Zs = filter(c, Z, d_lab_sw.get(), nullptr, 2);
      Bsr V;
      {
        Bsr SZ = spgemm(c, S, false, Zs, false, o.tau, LIF_FP64, 1.0, nullptr, 0.0, true);
        V = spgemm(c, Zs, true, SZ, false, o.tau, LIF_FP64, 1.0, nullptr, 0.0, true, false, o.sym_delta);
      }
      dn = axpby(c, -1.0, &V, 0.0, nullptr, 1.0, d_on_sw.get());
    }
    if (o.sym_delta) dn = mirror_upper(dn);
    Bsr keep = filter(c, delta, d_lab_keep.get(), nullptr, 2);
    delta = axpby(c, 1.0, &keep, 1.0, &dn, 0.0, nullptr);
    const std::vector<double> ss = node_sumsq(c, delta, d_rlo.get(), d_rhi.get(), nn);
    for (int s = 0; s < nn; ++s) {
      if (!sw[s]) continue;
      NodeState& ns = st[s];
      const double e = std::sqrt(ss[s]);
      ns.e_cur = ns.e_prev = ns.e = e;
      if (!ns.norms.empty()) ns.norms.back() = e;
      stale[s] = 0;
    }
  };
  if (!c.spec.sizes.get()) {
    c.spec.sizes = DBuf<int64_t>(c.pool, 2 * Ctx::Spec::kSlots);
    c.spec.overflow = DBuf<int>(c.pool, 1);
  }

  for (int k = 1;; ++k) {
    int n_active = 0;
    for (auto& s : st) n_active += s.active ? 1 : 0;
    if (n_active == 0) break;
    if (k > max_iter)
      throw Error(LIF_ERR_NO_CONVERGENCE, "refinement did not stop within max_iter = " + std::to_string(max_iter) +
                                              " iterations");
    if (labels_dirty) {
      std::fill(rowlab.begin(), rowlab.end(), -1);
      all_active = true;
      for (int s = 0; s < nn; ++s) {
        if (!st[s].active) {
          all_active = false;
          continue;
        }
        for (int i = bt.rlo[s]; i < bt.rhi[s]; ++i) rowlab[i] = s;
      }
      h2d(c, d_rowlab.get(), rowlab.data(), nb);
      labels_dirty = false;
    }
    // precision of each problem's correction in this iteration
    int n_red = 0, n_full = 0;
    for (int s = 0; s < nn; ++s) {
      red[s] = 0;
      if (!st[s].active) continue;
      red[s] = (o.prec != LIF_FP64 && (o.prec_switch <= 0.0 || st[s].e_cur > o.prec_switch)) ? 1 : 0;
      ++(red[s] ? n_red : n_full);
    }
    const bool split = n_red > 0 && n_full > 0;
    const int prec_it = n_red > 0 ? o.prec : LIF_FP64;
    if (split) {
      for (int i = 0; i < nb; ++i) {
        const int s = rowlab[i];
        lab_red[i] = (s >= 0 && red[s]) ? s : -1;
        lab_full[i] = (s >= 0 && !red[s]) ? s : -1;
      }
      if (!d_lab_red.get()) {
        d_lab_red = DBuf<int>(c.pool, nb);
        d_lab_full = DBuf<int>(c.pool, nb);
      }
      h2d(c, d_lab_red.get(), lab_red.data(), nb);
      h2d(c, d_lab_full.get(), lab_full.data(), nb);
    }
    // problems whose schedule moves to FP64 after reduced updates
    if (red_update) {
      std::vector<char> sw(nn, 0);
      bool any = false;
      for (int s = 0; s < nn; ++s) {
        sw[s] = st[s].active && stale[s] && !red[s];
        any = any || sw[s];
      }
      if (any) recompute_delta(sw);
    }
    // the delta update's inputs: FP32 (update_prec) for the problems in a
    // reduced iteration; with some problems in each precision the update
    // runs in two passes, each on its problems' part of M
    const int pu_all = (red_update && n_red > 0 && !split) ? o.update_prec : LIF_FP64;
    const bool upd_split = red_update && split;
    // One iteration.  After the first, every product is sized from the
    // previous iteration's counts (with a margin) instead of reading its
    // counts back; the counts and an overflow flag come back with the norms.
    // If a capacity was short the iteration is redone with exact sizes.
    // Sizing in advance saves a read-back per product, which only matters
    // for small products; an iteration whose products take more than a few
    // gigabytes reads its counts back (no margins, no redone work).
    const double blk_bytes = (double)S.b * S.b * sizeof(double);
    double caps_bytes = 0.0;
    for (const auto& cp : caps) caps_bytes += (double)cp[0] * blk_bytes + (double)cp[1] * sizeof(BlockPair);
    const bool carried = k == 1 && carry != nullptr;
    bool planned = o.presize != 0 && !caps.empty() && caps_split == split &&
                   caps_bytes <= (carried ? kPlanCarryBytes : kPlanIterBytes);
    Bsr Znew, dnew;
    std::vector<double> ss;
    bool big_iter = false;
    struct SpecOff {  // no sizing in advance outside this loop, also on errors
      Ctx& c;
      ~SpecOff() { c.spec.on = c.spec.record = c.spec.exact_large = false; }
    } spec_off{c};
    for (;;) {
      c.spec.on = planned;
      c.spec.record = !planned;
      c.spec.next = 0;
      c.spec.caps = caps;
      c.spec.seen.clear();
      c.spec.prec.clear();
      c.spec.exact.clear();
      if (planned) launch_fill_i32(c, c.spec.overflow.get(), 0, 1);
      // delta restricted to the problems still iterating
      Bsr dfilt;
      const bool restrict_rows = !all_active;
      if (restrict_rows) dfilt = filter(c, delta, d_rowlab.get(), nullptr, 2);
      const Bsr& da = restrict_rows ? dfilt : delta;

      // The products of one iteration are read only by the next product and
      // by the two sums, so their dropped blocks are left as null pointers
      // (holes) rather than compacted away.
      constexpr bool kHoles = true;
      // Two streams hold the iteration's buffers until its end; when the
      // products of the last iteration, or six matrices the size of Z, or
      // eight the size of delta would take more than a quarter of the GPU's
      // memory, the iteration runs on one stream, frees each buffer at once
      // and sizes its large products exactly.
      const double iter_bytes =
          std::max({caps_bytes, 6.0 * (double)Z.bound() * blk_bytes, 8.0 * (double)delta.bound() * blk_bytes});
      const double dev = (double)c.device_bytes();
      // (a panel size given in the options asks for this path too)
      const bool big = o.update_panel_rows > 0 || iter_bytes > 0.25 * dev ||
                       (double)c.pool->reserved() + iter_bytes > 0.5 * dev;
      c.spec.exact_large = big;
      big_iter = big;
      DeferFrees defer(c);
      if (big) defer.release();
      if (regular) {
        // Regular form (eq. refinement_nonlocal): P = b_m I, then
        // P <- b_j I + trunc(delta P) for j = m-1 .. 0, Z_{k+1} = trunc(Z P),
        // delta_{k+1} = I - trunc(trunc(Z_{k+1}^T S) Z_{k+1}).  P is kept as
        // X_j + b_j I with only X_j stored: delta P = delta X + b delta, the
        // scaled delta added to each output block before its truncation.
        // The first step has no product (X_m = 0): X_{m-1} = trunc(b_m delta).
        // Everything runs on the one stream: freed buffers are reusable at once.
        defer.release();
        Bsr X = spgemm(c, da, false, none, false, o.tau, LIF_FP64, 1.0, &da, bk[o.m], kHoles);
        for (int j = o.m - 2; j >= 0; --j)
          X = spgemm(c, da, false, X, false, o.tau, LIF_FP64, 1.0, &da, bk[j + 1], kHoles);
        // Z P = Z X_0 + b_0 Z; rows of finished problems (X_0 is empty there)
        // keep their blocks, which all passed the same truncation before
        Znew = spgemm(c, Z, false, X, false, o.tau, LIF_FP64, 1.0, &Z, bk[0]);
        X = Bsr();
        if (restrict_rows) {
          Bsr Zf = filter(c, Znew, d_rowlab.get(), nullptr, 2);
          dnew = regular_delta(c, S, Zf, o.tau, d_inb.get());
        } else {
          dnew = regular_delta(c, S, Znew, o.tau, d_inb.get());
        }
      } else {
      // M = Z sum_{k=1}^m b_k delta^k, Horner form, every product truncated:
      //   T_{m-1} = b_m delta + b_{m-1} I,  T_j = b_j I + trunc(delta T_{j+1}),
      //   q = trunc(delta T_1).
      // T_j is kept as X_j + c_j I with only X_j stored, so that the identity
      // is never formed: delta T = delta X + c delta, with the scaled delta
      // added to each output block before its truncation.  These products
      // run in the requested input precision (FP32 accumulation when
      // reduced), the delta-update below always in FP64.
      // the correction M on the rows of dd, with products in precision p
      auto correction = [&](const Bsr& dd, int p) {
        Bsr q;
        if (o.m == 1) {
          q = axpby(c, bk[1], &dd, 0.0, nullptr, 0.0, nullptr);
        } else {
          // first product: delta (b_m delta + b_{m-1} I) = b_m delta^2 + b_{m-1} delta
          // reduced precision: each Horner term is also written as the
          // transposed input-precision copy the next product reads
          const bool lp_out = p != LIF_FP64;
          Bsr X = spgemm(c, dd, false, dd, false, o.tau, p, bk[o.m], &dd, bk[o.m - 1], kHoles, lp_out);
          for (int j = o.m - 2; j >= 1; --j)
            X = spgemm(c, dd, false, X, false, o.tau, p, 1.0, &dd, bk[j], kHoles, lp_out);
          q = std::move(X);
        }
        return spgemm(c, Z, false, q, false, o.tau, p, 1.0, nullptr, 0.0, kHoles);
      };
      Bsr M, MR, MF;
      if (!split) {
        M = correction(da, prec_it);
      } else {
        // problems above the switch in reduced precision, the others in
        // FP64; Z is block diagonal, so the two parts of M share no row
        {
          Bsr dR = filter(c, delta, d_lab_red.get(), nullptr, 2);
          MR = correction(dR, o.prec);
        }
        {
          Bsr dF = filter(c, delta, d_lab_full.get(), nullptr, 2);
          MF = correction(dF, LIF_FP64);
        }
        M = axpby(c, 1.0, &MR, 1.0, &MF, 0.0, nullptr);
        if (!upd_split) {
          MR = Bsr();
          MF = Bsr();
        }
      }
      // delta_{k+1} = delta_k - Z_{k+1}^T (S M) - (S M)^T Z_k   (M^T S = (S M)^T)
      if (upd_split) {
        // the reduced problems' update with FP32 inputs, then the others' in
        // FP64: no problem has blocks in the other pass's products, so each
        // gets its own update (its rows pass the other sum unchanged)
        defer.release();
        Znew = axpby(c, 1.0, &Z, 1.0, &M, 0.0, nullptr);
        M = Bsr();
        Bsr d1 = update_pass(delta, MR, Z, Znew, planned, o.update_prec);
        MR = Bsr();
        dnew = update_pass(d1, MF, Z, Znew, planned, LIF_FP64);
        MF = Bsr();
      } else if (big) {
        // large products fill the GPU by themselves: one stream, and every
        // operand is released as soon as its last reader is queued
        Bsr SM = spgemm(c, S, false, M, false, o.tau, pu_all, 1.0, nullptr, 0.0, kHoles, pu_all != LIF_FP64);
        Znew = axpby(c, 1.0, &Z, 1.0, &M, 0.0, nullptr);
        M = Bsr();
        // panels of the update: as asked, or when its two products (about
        // delta's size each, half with a symmetric delta) would take more
        // than 1/16 of the memory, panels whose products take about 1/32
        int prow = o.update_panel_rows;
        if (prow == 0 && !planned) {
          const double upd = (o.sym_delta ? 1.0 : 2.0) * (double)delta.bound() * blk_bytes;
          if (upd > dev / 16.0) {
            const int np = (int)std::ceil(upd / (dev / 32.0));
            prow = (nb + np - 1) / np;
          }
        }
        if (prow > 0 && prow < nb) {
          dnew = delta_update_panels(delta, SM, Z, Znew, prow, pu_all);
          SM = Bsr();
        } else {
          Bsr X2 = spgemm(c, SM, true, Z, false, o.tau, pu_all, 1.0, nullptr, 0.0, kHoles, false, up);
          Bsr X1 = spgemm(c, Znew, true, SM, false, o.tau, pu_all, 1.0, nullptr, 0.0, kHoles, false, up);
          SM = Bsr();
          dnew = delta_update(X1, X2);
        }
        drop_update_copies(Z, Znew, pu_all);
      } else {
      // S M and then (S M)^T Z_k run on the side stream while Z + M and then
      // Z_{k+1}^T (S M) run on the main one; buffers freed meanwhile are
      // reused only after the synchronization at the end of the iteration.
      const hipStream_t main_s = c.stream, side_s = c.side_stream();
      c.stream_after(side_s, main_s);
      Bsr SM, X2;
      {
        StreamScope on_side(c, side_s);
        SM = spgemm(c, S, false, M, false, o.tau, pu_all, 1.0, nullptr, 0.0, kHoles, pu_all != LIF_FP64);
      }
      Znew = axpby(c, 1.0, &Z, 1.0, &M, 0.0, nullptr);
      c.stream_after(main_s, side_s);  // S M is complete
      {
        StreamScope on_side(c, side_s);
        X2 = spgemm(c, SM, true, Z, false, o.tau, pu_all, 1.0, nullptr, 0.0, kHoles, false, up);
      }
      Bsr X1 = spgemm(c, Znew, true, SM, false, o.tau, pu_all, 1.0, nullptr, 0.0, kHoles, false, up);
      c.stream_after(main_s, side_s);  // (S M)^T Z_k is complete
      M = Bsr();
      SM = Bsr();
      dnew = delta_update(X1, X2);
      X1 = Bsr();
      X2 = Bsr();
      }
      }

      const size_t nprod = planned ? c.spec.next : c.spec.seen.size();
      const std::vector<int> pprec = c.spec.prec;
      std::vector<std::array<int64_t, 2>> seen = c.spec.seen;
      c.spec.on = false;
      c.spec.record = false;
      int over = 0, nz_new = 0;
      std::vector<int64_t> sz(2 * nprod);
      std::vector<Ctx::Read> extra{{&nz_new, Znew.live(), sizeof(int)}};
      if (planned) {
        extra.push_back({&over, c.spec.overflow.get(), sizeof(int)});
        for (size_t i = 0; i < sz.size(); i += 8)
          extra.push_back({sz.data() + i, c.spec.sizes.get() + i, sizeof(int64_t) * std::min<size_t>(8, sz.size() - i)});
      }
      ss = node_sumsq(c, dnew, d_rlo.get(), d_rhi.get(), nn, extra);
      defer.release();  // both streams are idle: the main one waited for the side one
      Znew.nnzb = nz_new;
      if (planned && over) {
        ++c.stats.redone;
        planned = false;
        continue;
      }
      if (planned) {
        seen.clear();
        for (size_t i = 0; i < nprod; ++i) {
          const bool ex = i < c.spec.exact.size() && c.spec.exact[i][0] >= 0;  // sized exactly
          seen.push_back(ex ? c.spec.exact[i] : std::array<int64_t, 2>{sz[2 * i], sz[2 * i + 1]});
          const double fl = 2.0 * (double)S.b * S.b * S.b * (double)seen.back()[1];
          c.stats.products += seen.back()[1];
          count_symbolic(c, seen.back()[0], seen.back()[1], nb);
          c.stats.flops += fl;
          if (pprec[i] != LIF_FP64) c.stats.flops_lowp += fl;
          if (pprec[i] == LIF_MIXED_FP32) c.stats.flops_f32 += fl;
        }
      }
      // margins: output counts move little between iterations, block-product
      // counts can triple after the first iteration of a LIF level (delta_0
      // holds only the coupling blocks); pair slots are 16 bytes, and a
      // product over the planning limit is sized exactly anyway
      caps.clear();
      for (const auto& v : seen)
        caps.push_back(o.presize == 2 ? v : std::array<int64_t, 2>{v[0] + v[0] / 2 + 64, 4 * v[1] + 4096});
      break;
    }
    // Z_{k+1} and delta_{k+1} share the blocks they did not change with
    // Z_k, delta_k and the products; once the value arrays they keep alive
    // hold more than three times their own blocks (a quarter more on large
    // problems, where that memory is what limits the size), their blocks
    // are moved into one array (counts are known here: no extra read-back)
    const int64_t slack_num = big_iter ? 5 : 12, slack_den = 4;
    if (slack_den * Znew.store_blocks() > slack_num * Znew.nnzb + 256) Znew = compact_values(c, std::move(Znew));
    if (slack_den * dnew.store_blocks() > slack_num * dnew.nnzb + 256) dnew = compact_values(c, std::move(dnew));
    caps_split = split;
    if (carry && !split) *carry = caps;
    if (ck) ck->push_back(std::move(Z));  // Z_k is immutable: keep it, no copy
    Z = std::move(Znew);
    delta = std::move(dnew);
    if (verbose()) {
      double mx = 0.0;
      for (int s = 0; s < nn; ++s)
        if (st[s].active) mx = std::max(mx, std::sqrt(ss[s]));
      std::fprintf(stderr, "[lif] batch of %d problems, iteration %d: max ||delta||_F %.3e, Z %lld blocks, "
                   "delta %lld blocks (bound), %s stream(s), memory in use %.2f GiB, peak %.2f GiB, held %.2f GiB\n",
                   nn, k, mx, (long long)Z.nnzb, (long long)delta.bound(), big_iter ? "one" : "two",
                   c.pool->in_use() / 1073741824.0, c.pool->peak() / 1073741824.0,
                   c.pool->reserved() / 1073741824.0);
    }

    for (int s = 0; s < nn; ++s) {
      NodeState& ns = st[s];
      if (!ns.active) continue;
      const double e = std::sqrt(ss[s]);
      ns.iterations = k;
      ns.norms.push_back(e);
      if (red[s]) ++ns.reduced;
      stale[s] = red_update && red[s];
      const bool tested = !(o.prec_switch > 0.0 && red[s]);
      const Step d = stop_decision(k, e, ns.e_prev, ns.has_prev, o.m, o.stop, o.tol, &ns.stagnated, tested);
      ns.e_cur = e;
      if (d == Step::Diverged)
        throw Error(LIF_ERR_NO_CONVERGENCE, "refinement diverged: ||delta||_F = " + std::to_string(e) +
                                                " at iteration " + std::to_string(k) + " of problem " +
                                                std::to_string(s));
      ns.e = e;
      if (d == Step::Stop) {
        ns.active = false;
        labels_dirty = true;
      } else {
        ns.e_prev = e;
        ns.has_prev = true;
      }
    }
  }
}

}  // namespace

const unsigned char* all_rows_on(Ctx& c) {
  if (!c.ones.get()) {
    c.ones = DBuf<unsigned char>(c.pool, c.nb);
    LIF_HIP(hipMemsetAsync(c.ones.get(), 1, c.nb, c.stream));
  }
  return c.ones.get();
}

Plan make_plan(int64_t n, int b, int64_t base_rows) {
  Plan p;
  struct Item {
    int64_t lo, hi;
    int depth, parent;
    bool left;
  };
  std::vector<Item> stack{{0, n, 0, -1, false}};
  while (!stack.empty()) {
    Item it = stack.back();
    stack.pop_back();
    const int id = (int)p.nodes.size();
    p.nodes.push_back(PlanNode{it.lo, it.hi, it.depth});
    if (it.parent >= 0) {
      if (it.left)
        p.nodes[it.parent].left = id;
      else
        p.nodes[it.parent].right = id;
    }
    p.max_depth = std::max(p.max_depth, it.depth);
    if (it.hi - it.lo > base_rows) {
      const int64_t nbr = (it.hi - it.lo + b - 1) / b;
      const int64_t h = it.lo + ((nbr + 1) / 2) * b;
      stack.push_back({h, it.hi, it.depth + 1, id, false});
      stack.push_back({it.lo, h, it.depth + 1, id, true});
    }
  }
  return p;
}

Bsr run_irsi(Ctx& c, const Bsr& S, const Opts& o, RunInfo& info, Checkpoints* ck) {
  double cs = 0.0;
  if (o.start == LIF_START_GIVEN) {
    cs = o.start_value;
  } else if (o.start == LIF_START_INV_SQRT_LMAX) {
    cs = 1.0 / std::sqrt(o.start_value);
  } else {
    const double beta = gershgorin(c, S);
    cs = (o.start == LIF_START_SQRT2_OVER_GERSH) ? std::sqrt(2.0 / beta) : 1.0 / std::sqrt(beta);
  }
  LIF_REQUIRE(std::isfinite(cs) && cs > 0.0, LIF_ERR_INVALID, "start scale is not a positive finite number");
  info.start_scale = cs;
  const unsigned char* on = all_rows_on(c);
  Bsr Z = axpby(c, 0.0, nullptr, 0.0, nullptr, cs, on);
  // localized form: delta_0 = I - c^2 S by scaling; regular form: from the
  // truncated products like every later delta
  Bsr delta = o.refinement == LIF_REFINE_NONLOCAL ? regular_delta(c, S, Z, o.tau, on)
                                                   : axpby(c, -cs * cs, &S, 0.0, nullptr, 1.0, on);
  Batch bt;
  bt.nb = S.nb;
  bt.rlo = {0};
  bt.rhi = {S.nb};
  std::vector<NodeState> st;
  LevelCk* L = nullptr;
  if (ck) {
    ck->clear();
    ck->levels.emplace_back();
    L = &ck->levels.back();
    L->rlo = bt.rlo;
    L->rhi = bt.rhi;
  }
  refine_batch(c, S, Z, std::move(delta), bt, o, st, o.max_iter, L ? &L->Z : nullptr);
  if (L) {
    L->iters = {st[0].iterations};
    ck->valid = true;
  }
  info.iterations_top = st[0].iterations;
  info.iterations_total = st[0].iterations;
  info.iterations_reduced = st[0].reduced;
  info.stagnated = st[0].stagnated;
  info.delta_top = st[0].e;
  info.norms_top = st[0].norms;
  return Z;
}

Bsr run_refine_from(Ctx& c, const Bsr& S, Bsr&& Z0, const Opts& o, RunInfo& info) {
  const unsigned char* on = all_rows_on(c);
  Bsr delta;
  if (o.refinement == LIF_REFINE_NONLOCAL) {
    delta = regular_delta(c, S, Z0, o.tau, on);
  } else {
    Bsr SZ = spgemm(c, S, false, Z0, false, o.tau);
    Bsr ZSZ = spgemm(c, Z0, true, SZ, false, o.tau);
    SZ = Bsr();
    delta = axpby(c, -1.0, &ZSZ, 0.0, nullptr, 1.0, on);
  }
  Batch bt;
  bt.nb = S.nb;
  bt.rlo = {0};
  bt.rhi = {S.nb};
  std::vector<NodeState> st;
  Bsr Z = std::move(Z0);
  refine_batch(c, S, Z, std::move(delta), bt, o, st, o.max_iter);
  info.iterations_top = st[0].iterations;
  info.iterations_total = st[0].iterations;
  info.iterations_reduced = st[0].reduced;
  info.stagnated = st[0].stagnated;
  info.delta_top = st[0].e;
  info.norms_top = st[0].norms;
  return Z;
}

Bsr leaf_inverse_cholesky(Ctx& c, const Bsr& S, const std::vector<std::pair<int64_t, int64_t>>& ranges,
                          double tau) {
  const int b = S.b, nb = S.nb;
  const int nbase = (int)ranges.size();
  std::vector<int> blk0(nbase), nbbv(nbase), rowsv(nbase), base_of_row(nb, -1);
  std::vector<int64_t> tile0(nbase);
  int64_t tiles = 0;
  int max_nbb = 0;
  for (int s = 0; s < nbase; ++s) {
    blk0[s] = (int)(ranges[s].first / b);
    rowsv[s] = (int)(ranges[s].second - ranges[s].first);
    nbbv[s] = (rowsv[s] + b - 1) / b;
    tile0[s] = tiles;
    tiles += (int64_t)nbbv[s] * (nbbv[s] + 1) / 2;
    max_nbb = std::max(max_nbb, nbbv[s]);
    for (int i = 0; i < nbbv[s]; ++i) base_of_row[blk0[s] + i] = s;
  }
  DBuf<int> d_blk0(c.pool, nbase), d_nbb(c.pool, nbase), d_rows(c.pool, nbase), d_bor(c.pool, nb),
      d_err(c.pool, nbase);
  DBuf<int64_t> d_tile0(c.pool, nbase);
  h2d(c, d_blk0.get(), blk0.data(), nbase);
  h2d(c, d_nbb.get(), nbbv.data(), nbase);
  h2d(c, d_rows.get(), rowsv.data(), nbase);
  h2d(c, d_bor.get(), base_of_row.data(), nb);
  h2d(c, d_tile0.get(), tile0.data(), nbase);
  launch_fill_i32(c, d_err.get(), std::numeric_limits<int>::max(), nbase);
  DBuf<int> d_band(c.pool, 1);
  launch_fill_i32(c, d_band.get(), 0, 1);
  DBuf<unsigned char> nz(c.pool, (size_t)tiles);
  LIF_HIP(hipMemsetAsync(nz.get(), 0, (size_t)tiles, c.stream));

  const size_t tile_doubles = (size_t)b * b;
  DBuf<double> U(c.pool, (size_t)tiles * tile_doubles);
  Bsr Z;
  Z.n = S.n;
  Z.b = b;
  Z.nb = nb;
  // neither buffer is cleared: every tile of U that is read was scattered
  // from S or written in full by its first update, and every tile of Z is
  // written by potrf or trinv
  Store zs = new_store(c, tiles, b);
  {
    const int64_t snz = exact_nnzb(c, S);
    DBuf<int> rowof(c.pool, (size_t)std::max<int64_t>(snz, 1));
    launch_block_row_of(c, S.row_ptr.get(), nb, snz, rowof.get());
    launch_chol_scatter(c, rowof.get(), S.col.get(), S.ptrs(), snz, b, d_bor.get(), d_blk0.get(), d_nbb.get(),
                        d_tile0.get(), U.get(), nz.get(), d_band.get());
  }
  // tile band of S within the leaves: bounds the grids of trsm and update
  // and the first nonzero tile of each column of U
  int band = 0;
  c.d2h(&band, d_band.get(), sizeof(int));
  launch_chol_pad(c, nbase, d_nbb.get(), d_rows.get(), d_tile0.get(), b, U.get(), 1.0);
  // The factorization steps run on the main stream, one launch each.  Tile
  // column j of the inverse needs only columns < j and the V tiles of step
  // j, so it runs on the side stream as soon as step j is done, overlapping
  // the later (serial, small) factorization steps.
  hipStream_t side = c.side_stream();
  hipStream_t main_stream = c.stream;
  {
    // algorithmic flops of the band-limited factorization and the inverse:
    // per tile column k of a leaf with m = min(band, nbb - k - 1) tiles
    // beside the diagonal in the band: the diagonal tile's Cholesky and
    // inverse (b^3/3 each), the panel (m triangular-by-full products, b^3
    // each), the trailing update (m (m + 1) / 2 tile products, 2 b^3 each),
    // the tiles V of that column (min(band, k), b^3 each); then every tile
    // (i, j > i) of the inverse sums min(j - i, band) tile products
    const double b3 = (double)b * b * b;
    double fl = 0.0;
    for (int s = 0; s < nbase; ++s) {
      const int nbb = nbbv[s];
      for (int k = 0; k < nbb; ++k) {
        const double m = std::min(band, nbb - k - 1);
        fl += 2.0 * b3 / 3.0 + m * b3 + m * (m + 1.0) * b3 + std::min(band, k) * b3;
        for (int i = 0; i < k; ++i) fl += 2.0 * b3 * std::min(k - i, band);
      }
    }
    c.stats.leaf_flops += fl;
  }
  hipEvent_t leaf_t0 = c.timed_begin(2);
  // step 0's diagonal tile; every later one is factorized by the step before
  // (the workgroup of the last update it receives)
  launch_potrf(c, 0, nbase, d_nbb.get(), d_blk0.get(), d_tile0.get(), b, U.get(), zs->get(), nz.get(), d_err.get());
  // the inverse's columns go in pairs: a row's two tiles share most of
  // their operands (read once from HBM, then from L2)
  constexpr int kInvCols = 2;
  int next_col = 1;  // the first column of the inverse not yet launched
  for (int k = 0; k < max_nbb; ++k) {
    launch_step(c, k, band, nbase, max_nbb, d_nbb.get(), d_blk0.get(), d_tile0.get(), b, U.get(), zs->get(), nz.get(),
                d_err.get());
    if (k >= next_col && (k - next_col + 1 == kInvCols || k == max_nbb - 1)) {
      hipEvent_t ev = c.order_event((size_t)k);
      LIF_HIP(hipEventRecord(ev, main_stream));
      LIF_HIP(hipStreamWaitEvent(side, ev, 0));
      StreamScope on_side(c, side);
      launch_trinv(c, next_col, k - next_col + 1, band, nbase, d_nbb.get(), d_tile0.get(), b, U.get(), zs->get(),
                   nz.get());
      next_col = k + 1;
    }
  }
  {
    hipEvent_t ev = c.order_event(0);
    LIF_HIP(hipEventRecord(ev, side));
    LIF_HIP(hipStreamWaitEvent(main_stream, ev, 0));
  }
  c.timed_end(leaf_t0, Ctx::Leaf);  // the steps and the inverse's columns on the second stream
  launch_chol_pad(c, nbase, d_nbb.get(), d_rows.get(), d_tile0.get(), b, zs->get(), 0.0);
  std::vector<int> err(nbase);
  c.d2h(err.data(), d_err.get(), nbase * sizeof(int));
  for (int s = 0; s < nbase; ++s)
    if (err[s] != std::numeric_limits<int>::max())
      throw Error(LIF_ERR_NOT_PD, "leaf " + std::to_string(s) + " (rows " + std::to_string(ranges[s].first) + ".." +
                                      std::to_string(ranges[s].second) + "): non-positive pivot at row " +
                                      std::to_string(err[s]));
  // block-CSR view of the packed tiles: row I of leaf s holds columns I..end
  std::vector<int> rp(nb + 1, 0), col;
  col.reserve((size_t)tiles);
  for (int I = 0; I < nb; ++I) {
    const int s = base_of_row[I];
    if (s >= 0) {
      const int end = blk0[s] + nbbv[s];
      for (int J = I; J < end; ++J) col.push_back(J);
    }
    rp[I + 1] = (int)col.size();
  }
  LIF_REQUIRE((int64_t)col.size() == tiles, LIF_ERR_INVALID, "leaf ranges do not cover whole block rows");
  Z.nnzb = tiles;
  Z.cap = tiles;
  Z.row_ptr = DBuf<int>(c.pool, nb + 1);
  Z.col = DBuf<int>(c.pool, (size_t)tiles);
  h2d(c, Z.row_ptr.get(), rp.data(), nb + 1);
  h2d(c, Z.col.get(), col.data(), (size_t)tiles);
  Z.blk = DBuf<const double*>(c.pool, (size_t)tiles);
  Z.store.push_back(zs);
  launch_fill_ptrs(c, Z.blk.get(), zs->get(), b, tiles);
  // leaf truncation (Sec. 5); exactly-zero tiles of the triangle are dropped
  // as well (the smallest positive double as threshold at tau = 0)
  DBuf<double> nrm = block_norms(c, Z);
  Bsr Zt = truncate(c, std::move(Z), nrm.get(), std::max(tau, std::numeric_limits<double>::denorm_min()));
  // the packed triangles hold every tile of each leaf; keep only the kept ones
  Bsr out = compact_values(c, std::move(Zt));
  task_after(c, out, false, {&S});  // one factorization task for all leaves of the batch
  return out;
}

namespace {

// One node of the recursive inverse Cholesky (Alg. 1) on rows [lo, hi) of
// Sn (global coordinates; Sn holds no block outside the range):
//   Z00 = rinch(S00), R = trunc(Z00^T S01), Q = S11 - trunc(R^T R),
//   Z11 = rinch(Q), Z01 = -trunc(trunc(Z00 R) Z11), Z10 = 0;
// ranges of at most base_rows rows are leaves (truncated inverse Cholesky).
// The split is LIF's (the leading ceil(nb/2) blocks).  Q's rows depend on
// Z00, so the two halves run one after the other.
Bsr rinch_node(Ctx& c, const Bsr& Sn, int64_t lo, int64_t hi, const Opts& o, int depth, RunInfo& info) {
  info.levels = std::max(info.levels, depth + 1);
  const int b = Sn.b, nb = Sn.nb;
  if (hi - lo <= o.base_rows) return leaf_inverse_cholesky(c, Sn, {{lo, hi}}, o.tau);
  const int64_t nbr = (hi - lo + b - 1) / b;
  const int64_t mid = lo + ((nbr + 1) / 2) * b;
  // block-row labels: 0 = leading part, 1 = trailing part, -1 = elsewhere
  std::vector<int> lab(nb, -1), lab0(nb, -1), lab1(nb, -1);
  const int r0 = (int)(lo / b), rm = (int)(mid / b), r1 = (int)((hi + b - 1) / b);
  for (int i = r0; i < r1; ++i) {
    lab[i] = i < rm ? 0 : 1;
    (i < rm ? lab0 : lab1)[i] = 0;
  }
  DBuf<int> d_lab(c.pool, nb), d_lab0(c.pool, nb), d_lab1(c.pool, nb);
  h2d(c, d_lab.get(), lab.data(), nb);
  h2d(c, d_lab0.get(), lab0.data(), nb);
  h2d(c, d_lab1.get(), lab1.data(), nb);
  Bsr S00 = filter(c, Sn, d_lab0.get(), d_lab0.get(), 0);
  Bsr S01 = filter(c, Sn, d_lab.get(), d_lab.get(), 1);
  Bsr S11 = filter(c, Sn, d_lab1.get(), d_lab1.get(), 0);
  c.sync();  // the label vectors go out of scope
  Bsr Z00 = rinch_node(c, S00, lo, mid, o, depth + 1, info);
  S00 = Bsr();
  Bsr R = spgemm(c, Z00, true, S01, false, o.tau);
  S01 = Bsr();
  Bsr Q;
  {
    Bsr RtR = spgemm(c, R, true, R, false, o.tau);
    Q = axpby(c, 1.0, &S11, -1.0, &RtR, 0.0, nullptr);  // the difference is not truncated
  }
  S11 = Bsr();
  Bsr Z11 = rinch_node(c, Q, mid, hi, o, depth + 1, info);
  Q = Bsr();
  Bsr Z01;
  {
    Bsr T = spgemm(c, Z00, false, R, false, o.tau);
    Z01 = spgemm(c, T, false, Z11, false, o.tau, LIF_FP64, -1.0);
  }
  return axpby3(c, 1.0, &Z00, 1.0, &Z01, 1.0, &Z11);  // disjoint parts: every block shared
}

}  // namespace

Bsr run_rinch(Ctx& c, const Bsr& S, const Opts& o, RunInfo& info) {
  info.levels = 0;
  info.iterations_total = 0;
  info.iterations_top = 0;
  return rinch_node(c, S, 0, S.n, o, 0, info);
}

Bsr run_lif(Ctx& c, const Bsr& S, const Opts& o, RunInfo& info, Checkpoints* ck) {
  const int b = S.b, nb = S.nb;
  const Plan plan = make_plan(S.n, b, o.base_rows);
  std::vector<std::pair<int64_t, int64_t>> leaves;
  for (const auto& nd : plan.nodes)
    if (nd.left < 0) leaves.emplace_back(nd.lo, nd.hi);
  std::sort(leaves.begin(), leaves.end());
  Bsr Z = leaf_inverse_cholesky(c, S, leaves, o.tau);
  if (ck) {
    ck->clear();
    ck->lif = true;
    ck->Z_leaf = copy(c, Z);
  }
  info.levels = 0;
  info.iterations_total = 0;
  // every level's refinement runs the same sequence of products; each
  // level starts from the capacities the level below ended with
  std::vector<std::array<int64_t, 2>> carry, setup_caps;
  for (int d = plan.max_depth - 1; d >= 0; --d) {
    std::vector<int> ids;
    for (int i = 0; i < (int)plan.nodes.size(); ++i)
      if (plan.nodes[i].depth == d && plan.nodes[i].left >= 0) ids.push_back(i);
    if (ids.empty()) continue;
    std::sort(ids.begin(), ids.end(), [&](int a, int x) { return plan.nodes[a].lo < plan.nodes[x].lo; });
    const int nn = (int)ids.size();
    Batch bt;
    bt.nb = nb;
    std::vector<int> lab(nb, -1), side(nb, -1);
    for (int s = 0; s < nn; ++s) {
      const PlanNode& nd = plan.nodes[ids[s]];
      const int r0 = (int)(nd.lo / b), r1 = (int)((nd.hi + b - 1) / b);
      const int rm = (int)(plan.nodes[nd.left].hi / b);
      bt.rlo.push_back(r0);
      bt.rhi.push_back(r1);
      for (int i = r0; i < r1; ++i) {
        lab[i] = s;
        side[i] = 2 * s + (i >= rm ? 1 : 0);
      }
    }
    DBuf<int> d_lab(c.pool, nb), d_side(c.pool, nb);
    h2d(c, d_lab.get(), lab.data(), nb);
    h2d(c, d_side.get(), side.data(), nb);
    // the level's diagonal problems, and the couplings B of each split
    Bsr S_lvl = filter(c, S, d_lab.get(), d_lab.get(), 0);
    const bool regular = o.refinement == LIF_REFINE_NONLOCAL;
    Bsr S_up = regular ? Bsr() : filter(c, S, d_side.get(), d_side.get(), 1);
    // Localized form: delta_0 = -[[0, X], [X^T, 0]], X = (Z_A^T B) Z_C.  The
    // two products are sized in advance from the level below (their counts and an
    // overflow flag come back with delta_0's norms; a short capacity redoes
    // them with exact sizes).
    Bsr delta0;
    std::vector<double> ss0;
    std::vector<unsigned char> inb;
    DBuf<unsigned char> d_inb;
    if (regular) {
      // recursive inverse factorization with the regular correction
      // (Sec. 2.3): delta_0 = I - (Z_0^T S) Z_0 on the level's rows
      inb.resize(nb);
      for (int i = 0; i < nb; ++i) inb[i] = lab[i] >= 0 ? 1 : 0;
      d_inb = DBuf<unsigned char>(c.pool, nb);
      h2d(c, d_inb.get(), inb.data(), nb);
      delta0 = regular_delta(c, S_lvl, Z, o.tau, d_inb.get());
    } else {
      DBuf<int> d_rlo(c.pool, nn), d_rhi(c.pool, nn);
      h2d(c, d_rlo.get(), bt.rlo.data(), nn);
      h2d(c, d_rhi.get(), bt.rhi.data(), nn);
      if (!c.spec.sizes.get()) {
        c.spec.sizes = DBuf<int64_t>(c.pool, 2 * Ctx::Spec::kSlots);
        c.spec.overflow = DBuf<int>(c.pool, 1);
      }
      double setup_bytes = 0.0;
      for (const auto& cp : setup_caps)
        setup_bytes += (double)cp[0] * b * b * sizeof(double) + (double)cp[1] * sizeof(BlockPair);
      for (bool planned = o.presize != 0 && !setup_caps.empty() && setup_bytes <= kPlanCarryBytes;;
           planned = false) {
        struct SpecOff {
          Ctx& c;
          ~SpecOff() { c.spec.on = c.spec.record = c.spec.exact_large = false; }
        } spec_off{c};
        c.spec.on = planned;
        c.spec.record = !planned;
        c.spec.next = 0;
        c.spec.caps = setup_caps;
        c.spec.seen.clear();
        c.spec.prec.clear();
        c.spec.exact.clear();
        // large levels: the two products are sized exactly once they are large
        const double zb = 4.0 * (double)Z.bound() * b * b * sizeof(double), dev = (double)c.device_bytes();
        c.spec.exact_large = zb > 0.25 * dev || (double)c.pool->reserved() + zb > 0.5 * dev;
        if (planned) launch_fill_i32(c, c.spec.overflow.get(), 0, 1);
        Bsr W = spgemm(c, Z, true, S_up, false, o.tau);
        Bsr X = spgemm(c, W, false, Z, false, o.tau);
        W = Bsr();
        Bsr Xt = transpose(c, X);
        delta0 = axpby(c, -1.0, &X, -1.0, &Xt, 0.0, nullptr);
        c.spec.on = c.spec.record = false;
        int over = 0;
        int64_t sz[4] = {0, 0, 0, 0};
        std::vector<Ctx::Read> extra;
        if (planned) {
          extra.push_back({&over, c.spec.overflow.get(), sizeof(int)});
          extra.push_back({sz, c.spec.sizes.get(), sizeof(sz)});
        }
        ss0 = node_sumsq(c, delta0, d_rlo.get(), d_rhi.get(), nn, extra);
        if (planned && over) {
          ++c.stats.redone;
          continue;
        }
        std::vector<std::array<int64_t, 2>> seen = c.spec.seen;
        if (planned) {
          seen = {{sz[0], sz[1]}, {sz[2], sz[3]}};
          for (size_t i = 0; i < seen.size(); ++i) {
            if (i < c.spec.exact.size() && c.spec.exact[i][0] >= 0) seen[i] = c.spec.exact[i];  // sized exactly
            const double fl = 2.0 * (double)S.b * S.b * S.b * (double)seen[i][1];
            c.stats.products += seen[i][1];
            count_symbolic(c, seen[i][0], seen[i][1], nb);
            c.stats.flops += fl;
          }
        }
        setup_caps.clear();
        for (const auto& v : seen) setup_caps.push_back({v[0] + v[0] / 2 + 64, 4 * v[1] + 4096});
        break;
      }
    }
    S_up = Bsr();
    std::vector<NodeState> st;
    LevelCk* L = nullptr;
    if (ck) {
      ck->levels.emplace(ck->levels.begin());  // top level first
      L = &ck->levels.front();
      L->rlo = bt.rlo;
      L->rhi = bt.rhi;
      // parts after the split: children of this depth's nodes, and every
      // other row keeps the leaf or node it belongs to at this stage
      L->part_lab.assign(nb, -1);
      int next = 0;
      for (int s = 0; s < nn; ++s)
        for (int i = bt.rlo[s]; i < bt.rhi[s]; ++i) L->part_lab[i] = 2 * s + (side[i] & 1);
      next = 2 * nn;
      for (const auto& nd : plan.nodes) {
        const bool part = (nd.depth == d + 1) || (nd.left < 0 && nd.depth <= d);
        if (!part) continue;
        const int r0 = (int)(nd.lo / b), r1 = (int)((nd.hi + b - 1) / b);
        if (L->part_lab[r0] >= 0) continue;  // a child of this depth, labelled above
        for (int i = r0; i < r1; ++i) L->part_lab[i] = next;
        ++next;
      }
    }
    refine_batch(c, S_lvl, Z, std::move(delta0), bt, o, st, o.max_iter, L ? &L->Z : nullptr,
                 o.presize != 0 ? &carry : nullptr, regular ? nullptr : &ss0);
    if (L) {
      for (auto& ns : st) L->iters.push_back(ns.iterations);
      L->S_lvl = std::move(S_lvl);
    }
    info.levels += 1;
    for (auto& ns : st) {
      info.iterations_total += ns.iterations;
      info.iterations_reduced += ns.reduced;
    }
    if (d == 0) {
      info.iterations_top = st[0].iterations;
      info.stagnated = st[0].stagnated;
      info.delta_top = st[0].e;
      info.norms_top = st[0].norms;
    }
    c.sync();  // label vectors go out of scope
  }
  if (ck) ck->valid = true;
  return Z;
}

double residual(Ctx& c, const Bsr& S, const Bsr& Z, int panel_rows) {
  // R = I - Z^T (S Z), untruncated, with ||R||_F^2 summed over panels of
  // R's block columns: columns [p0, p1) of R, taken as the rows of their
  // transpose (S Z_p)^T Z, Z_p the block columns of Z in [p0, p1), so neither
  // S Z nor R is ever held whole and the transposed operand is the panel's
  // S Z_p, not Z (a transpose has the Frobenius norm of its matrix).
  // Automatic panels: one, unless R could take more than min(8 GiB, 1/16 of
  // the device memory the handle may use).
  const double kPanelBytes = std::min(8.0 * double(1u << 30), (double)c.device_bytes() / 16.0);
  const int nb = S.nb;
  const double row_bytes = (double)nb * S.b * S.b * sizeof(double);  // a dense block column of R
  const int rows = panel_rows > 0 ? std::min(panel_rows, nb)
                                  : (int)std::max(1.0, std::min((double)nb, std::floor(kPanelBytes / row_bytes)));
  Bsr SZ;
  if (rows >= nb) SZ = spgemm(c, S, false, Z, false, 0.0);
  // host sources of asynchronous copies, rewritten only after the
  // read-back that ends each panel
  std::vector<int> zeros(nb, 0), clab(nb), lo(1), hi(1);
  std::vector<unsigned char> on(nb);
  DBuf<int> d_zeros(c.pool, nb), d_clab(c.pool, nb), d_lo(c.pool, 1), d_hi(c.pool, 1);
  DBuf<unsigned char> d_on(c.pool, nb);
  h2d(c, d_zeros.get(), zeros.data(), nb);
  double ss = 0.0;
  lo[0] = 0;
  hi[0] = nb;
  h2d(c, d_lo.get(), lo.data(), 1);
  h2d(c, d_hi.get(), hi.data(), 1);
  for (int p0 = 0; p0 < nb; p0 += rows) {
    const int p1 = std::min(nb, p0 + rows);
    Bsr R;
    if (rows >= nb) {
      Bsr ZSZ = spgemm(c, Z, true, SZ, false, 0.0);
      R = axpby(c, -1.0, &ZSZ, 0.0, nullptr, 1.0, all_rows_on(c));
    } else {
      for (int j = 0; j < nb; ++j) {
        clab[j] = (j >= p0 && j < p1) ? 0 : -1;
        on[j] = (j >= p0 && j < p1) ? 1 : 0;
      }
      h2d(c, d_clab.get(), clab.data(), nb);
      h2d(c, d_on.get(), on.data(), nb);
      Bsr P;
      {
        Bsr SZp;
        {
          Bsr Zp = filter(c, Z, d_zeros.get(), d_clab.get(), 0);
          SZp = spgemm(c, S, false, Zp, false, 0.0);
        }
        P = spgemm(c, SZp, true, Z, false, 0.0);
      }
      // the identity's blocks (j, j) with j in the panel
      R = axpby(c, -1.0, &P, 0.0, nullptr, 1.0, d_on.get());
    }
    ss += node_sumsq(c, R, d_lo.get(), d_hi.get(), 1)[0];
  }
  return std::sqrt(ss);
}

}  // namespace lif
