// C ABI entry points (include/lif.h): validation, handle ownership, status
// codes.  No exception crosses this boundary.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <new>

#include "driver.h"

using namespace lif;

struct lif_handle_s {
  Opts opts;
  Pool pool;
  Ctx ctx;
  Bsr S;
  Bsr Z;
  bool has_Z = false;
  Checkpoints ck;
  Bsr dS;
  bool has_dS = false;
  std::string err;
  explicit lif_handle_s(uint64_t cap) : pool(cap) {}
};

namespace {

thread_local std::string g_create_error;

void validate_opts(const lif_opts& o) {
  LIF_REQUIRE(o.m >= 1 && o.m <= 8, LIF_ERR_INVALID, "opts.m must be in 1..8");
  LIF_REQUIRE(std::isfinite(o.tau) && o.tau >= 0.0, LIF_ERR_INVALID, "opts.tau must be finite and >= 0");
  LIF_REQUIRE(o.prec == LIF_FP64 || o.prec == LIF_MIXED_FP32 || o.prec == LIF_MIXED_BF16, LIF_ERR_INVALID,
              "opts.prec is invalid");
  LIF_REQUIRE(o.stop == LIF_STOP_PAPER || o.stop == LIF_STOP_TOL, LIF_ERR_INVALID, "opts.stop is invalid");
  LIF_REQUIRE(std::isfinite(o.tol) && o.tol >= 0.0, LIF_ERR_INVALID, "opts.tol must be finite and >= 0");
  LIF_REQUIRE(o.max_iter >= 1 && o.max_iter <= 10000, LIF_ERR_INVALID, "opts.max_iter must be in 1..10000");
  LIF_REQUIRE(o.presize >= 0 && o.presize <= 2, LIF_ERR_INVALID, "opts.presize must be 0, 1 or 2");
  LIF_REQUIRE(o.start >= 0 && o.start <= 3, LIF_ERR_INVALID, "opts.start is invalid");
  LIF_REQUIRE(o.refinement == LIF_REFINE_LOCAL || o.refinement == LIF_REFINE_NONLOCAL, LIF_ERR_INVALID,
              "opts.refinement is invalid");
  LIF_REQUIRE(o.refinement == LIF_REFINE_LOCAL || o.prec == LIF_FP64, LIF_ERR_INVALID,
              "opts.refinement = LIF_REFINE_NONLOCAL needs prec = LIF_FP64");
  LIF_REQUIRE(std::isfinite(o.prec_switch) && o.prec_switch >= 0.0, LIF_ERR_INVALID,
              "opts.prec_switch must be finite and >= 0");
  LIF_REQUIRE(o.sym_delta == 0 || o.sym_delta == 1, LIF_ERR_INVALID, "opts.sym_delta must be 0 or 1");
  LIF_REQUIRE(o.residual_panel_rows >= 0, LIF_ERR_INVALID, "opts.residual_panel_rows must be >= 0");
  LIF_REQUIRE(o.update_panel_rows >= 0, LIF_ERR_INVALID, "opts.update_panel_rows must be >= 0");
  LIF_REQUIRE(o.timing >= 0 && o.timing <= 2, LIF_ERR_INVALID, "opts.timing must be 0, 1 or 2");
  LIF_REQUIRE(o.update_prec == LIF_FP64 || o.update_prec == LIF_MIXED_FP32, LIF_ERR_INVALID,
              "opts.update_prec must be LIF_FP64 or LIF_MIXED_FP32");
  if (o.update_prec != LIF_FP64) {
    LIF_REQUIRE(o.prec != LIF_FP64 && o.prec_switch > 0.0, LIF_ERR_INVALID,
                "opts.update_prec = LIF_MIXED_FP32 needs a reduced prec with prec_switch > 0");
    LIF_REQUIRE(o.checkpoint == 0, LIF_ERR_INVALID, "opts.update_prec = LIF_MIXED_FP32 needs checkpoint = 0");
  }
  if (o.start == LIF_START_INV_SQRT_LMAX || o.start == LIF_START_GIVEN)
    LIF_REQUIRE(std::isfinite(o.start_value) && o.start_value > 0.0, LIF_ERR_INVALID,
                "opts.start_value must be > 0 for this start");
}

// Host copy of the index arrays of a block list (device lists are copied down).
struct HostIndex {
  std::vector<int32_t> r, c;
};

HostIndex host_index(const lif_blocks& B) {
  HostIndex h;
  h.r.resize((size_t)B.nnzb);
  h.c.resize((size_t)B.nnzb);
  if (B.nnzb == 0) return h;
  if (B.on_device) {
    LIF_HIP(hipMemcpy(h.r.data(), B.brow, B.nnzb * sizeof(int32_t), hipMemcpyDeviceToHost));
    LIF_HIP(hipMemcpy(h.c.data(), B.bcol, B.nnzb * sizeof(int32_t), hipMemcpyDeviceToHost));
  } else {
    std::copy(B.brow, B.brow + B.nnzb, h.r.begin());
    std::copy(B.bcol, B.bcol + B.nnzb, h.c.begin());
  }
  return h;
}

// Checks a block list: shape, sorted unique in-range coordinates, zero
// padding beyond n; optionally a symmetric block pattern.
void check_blocks(const lif_blocks* B, bool need_symmetric, const char* what) {
  const std::string w(what);
  LIF_REQUIRE(B != nullptr, LIF_ERR_INVALID, w + ": null block list");
  LIF_REQUIRE(B->n > 0, LIF_ERR_INVALID, w + ": n must be > 0");
  LIF_REQUIRE(B->b == 32 || B->b == 64, LIF_ERR_INVALID, w + ": b must be 32 or 64");
  const int64_t nb = (B->n + B->b - 1) / B->b;
  LIF_REQUIRE(nb <= 32768, LIF_ERR_INVALID, w + ": more than 32768 block rows");
  LIF_REQUIRE(B->nnzb >= 0 && B->nnzb <= nb * nb && B->nnzb < (int64_t)1 << 31, LIF_ERR_INVALID,
              w + ": nnzb out of range");
  LIF_REQUIRE(B->nnzb == 0 || (B->brow && B->bcol && B->vals), LIF_ERR_INVALID, w + ": null array");
  HostIndex h = host_index(*B);
  for (int64_t e = 0; e < B->nnzb; ++e) {
    LIF_REQUIRE(h.r[e] >= 0 && h.r[e] < nb && h.c[e] >= 0 && h.c[e] < nb, LIF_ERR_INVALID,
                w + ": block coordinate out of range at entry " + std::to_string(e));
    if (e)
      LIF_REQUIRE(h.r[e] > h.r[e - 1] || (h.r[e] == h.r[e - 1] && h.c[e] > h.c[e - 1]), LIF_ERR_INVALID,
                  w + ": blocks not sorted by (row, col) or duplicated at entry " + std::to_string(e));
  }
  if (need_symmetric) {
    std::vector<int64_t> rp(nb + 1, 0);
    for (int64_t e = 0; e < B->nnzb; ++e) rp[h.r[e] + 1]++;
    for (int64_t i = 0; i < nb; ++i) rp[i + 1] += rp[i];
    for (int64_t e = 0; e < B->nnzb; ++e) {
      const int32_t i = h.r[e], j = h.c[e];
      const auto lo = h.c.begin() + rp[j], hi = h.c.begin() + rp[j + 1];
      LIF_REQUIRE(std::binary_search(lo, hi, i), LIF_ERR_INVALID,
                  w + ": block pattern not symmetric: (" + std::to_string(i) + "," + std::to_string(j) +
                      ") present, mirror missing");
    }
  }
  // padding of the last block row / column must be zero
  const int tail = (int)(B->n - (nb - 1) * B->b);
  if (tail != B->b) {
    const size_t bb = (size_t)B->b * B->b;
    std::vector<double> blk(bb);
    for (int64_t e = 0; e < B->nnzb; ++e) {
      if (h.r[e] != nb - 1 && h.c[e] != nb - 1) continue;
      if (B->on_device)
        LIF_HIP(hipMemcpy(blk.data(), B->vals + e * bb, bb * sizeof(double), hipMemcpyDeviceToHost));
      else
        std::copy(B->vals + e * bb, B->vals + (e + 1) * bb, blk.begin());
      for (int r = 0; r < B->b; ++r)
        for (int c = 0; c < B->b; ++c) {
          const bool pad = (h.r[e] == nb - 1 && r >= tail) || (h.c[e] == nb - 1 && c >= tail);
          LIF_REQUIRE(!pad || blk[(size_t)r * B->b + c] == 0.0, LIF_ERR_INVALID,
                      w + ": nonzero entry beyond n in block " + std::to_string(e));
        }
    }
  }
}

template <typename F>
lif_status guarded(lif_handle h, F&& f) {
  try {
    if (h) h->err.clear();
    f();
    return LIF_OK;
  } catch (const Error& e) {
    if (h) h->err = e.what();
    return e.status;
  } catch (const std::bad_alloc&) {
    if (h) h->err = "host allocation failed";
    return LIF_ERR_OUT_OF_MEMORY;
  } catch (const std::exception& e) {
    if (h) h->err = e.what();
    return LIF_ERR_INVALID;
  } catch (...) {
    if (h) h->err = "unknown failure";
    return LIF_ERR_INVALID;
  }
}

// The options of a handle from the caller's struct (the cap is the pool's).
void copy_opts(lif_handle h, const lif_opts& o) {
  Opts& p = h->opts;
  p.m = o.m;
  p.tau = o.tau;
  p.prec = o.prec;
  p.stop = o.stop;
  p.tol = o.tol;
  p.max_iter = o.max_iter;
  p.base_rows = o.base_rows;
  p.start = o.start;
  p.start_value = o.start_value;
  p.checkpoint = o.checkpoint != 0;
  p.presize = o.presize;
  p.refinement = o.refinement;
  p.prec_switch = o.prec_switch;
  p.sym_delta = o.sym_delta != 0;
  p.residual_panel_rows = o.residual_panel_rows;
  p.update_panel_rows = o.update_panel_rows;
  p.update_prec = o.update_prec;
  h->ctx.stream = static_cast<hipStream_t>(o.stream);
  h->ctx.timing = o.timing != 0;
  h->ctx.timing_level = o.timing;
}

void fill_info(lif_handle h, const RunInfo& ri, double seconds, lif_info* info) {
  if (!info) return;
  h->ctx.flush_timing();
  std::memset(info, 0, sizeof(*info));
  info->iterations_top = ri.iterations_top;
  info->levels = ri.levels;
  info->iterations_total = ri.iterations_total;
  info->stagnated = ri.stagnated ? 1 : 0;
  info->start_scale = ri.start_scale;
  info->delta_tracked = ri.delta_top;
  info->flops_leaf_gemm = h->ctx.stats.flops;
  info->seconds_total = seconds;
  info->seconds_leaf_gemm = h->ctx.stats.gemm_ms * 1e-3;
  info->leaf_gemm_launches = h->ctx.stats.gemm_launches;
  info->products_total = h->ctx.stats.products;
  info->cpl_tasks = h->ctx.stats.cpl;
  info->cpl_products = h->ctx.stats.cpl_products;
  info->iterations_reduced = ri.iterations_reduced;
  info->mem_peak_bytes = h->pool.peak();
  info->mem_reserved_bytes = h->pool.reserved();
  info->products_compacted = (int32_t)h->ctx.stats.compacted;
  info->pair_panels = (int32_t)h->ctx.stats.panels;
  info->nnzb_Z = h->has_Z ? exact_nnzb(h->ctx, h->Z) : 0;
  info->n_norms = (int32_t)std::min<size_t>(64, ri.norms_top.size());
  for (int k = 0; k < info->n_norms; ++k) info->norms[k] = ri.norms_top[k];
  info->iterations_redone = h->ctx.stats.redone;
  info->flops_leaf_gemm_reduced = h->ctx.stats.flops_lowp;
  info->seconds_leaf_gemm_reduced = h->ctx.stats.gemm_ms_lowp * 1e-3;
  info->leaf_gemm_launches_reduced = h->ctx.stats.gemm_launches_lowp;
  info->flops_leaf_gemm_fp32 = h->ctx.stats.flops_f32;
  info->seconds_leaf_gemm_fp32 = h->ctx.stats.gemm_ms_f32 * 1e-3;
  info->leaf_gemm_launches_fp32 = h->ctx.stats.gemm_launches_f32;
  info->seconds_leaf_factorization = h->ctx.stats.leaf_ms * 1e-3;
  info->flops_leaf_factorization = h->ctx.stats.leaf_flops;
  info->seconds_symbolic = h->ctx.stats.sym_ms * 1e-3;
  info->bytes_symbolic = h->ctx.stats.sym_bytes;
  info->symbolic_launches = h->ctx.stats.sym_launches;
}

void reset_stats(lif_handle h) {
  h->ctx.flush_timing();
  h->ctx.stats = Stats();
  h->pool.reset_peak();
}

lif_status copy_out(lif_handle h, const Bsr& A, int64_t* nnzb, int32_t* brow, int32_t* bcol, double* vals,
                    int32_t on_device) {
  LIF_REQUIRE(nnzb != nullptr, LIF_ERR_INVALID, "nnzb is null");
  const int64_t have = exact_nnzb(h->ctx, A);
  if (brow == nullptr) {
    *nnzb = have;
    return LIF_OK;
  }
  LIF_REQUIRE(*nnzb >= have, LIF_ERR_INVALID,
              "output capacity " + std::to_string(*nnzb) + " < " + std::to_string(have) + " blocks");
  LIF_REQUIRE(have == 0 || (bcol && vals), LIF_ERR_INVALID, "null output array");
  bsr_to_blocks(h->ctx, A, brow, bcol, vals, on_device != 0);
  *nnzb = have;
  return LIF_OK;
}

}  // namespace

namespace lif {
void validate_blocks(const lif_blocks* B, bool need_symmetric, const char* what) {
  check_blocks(B, need_symmetric, what);
}
void set_thread_error(const std::string& msg) { g_create_error = msg; }
}  // namespace lif

extern "C" {

lif_status lif_opts_default(lif_opts* o) {
  if (!o) return LIF_ERR_INVALID;
  std::memset(o, 0, sizeof(*o));
  o->m = 4;
  o->tau = 0.0;
  o->prec = LIF_FP64;
  o->stop = LIF_STOP_PAPER;
  o->tol = 1e-10;
  o->max_iter = 100;
  o->base_rows = 4096;
  o->start = LIF_START_SQRT2_OVER_GERSH;
  o->start_value = 0.0;
  o->checkpoint = 0;
  o->mem_cap_bytes = 0;
  o->stream = nullptr;
  o->timing = 0;
  o->presize = 1;
  o->refinement = LIF_REFINE_LOCAL;
  o->prec_switch = 0.0;
  o->sym_delta = 0;
  o->residual_panel_rows = 0;
  o->update_panel_rows = 0;
  o->update_prec = LIF_FP64;
  return LIF_OK;
}

lif_status lif_create(const lif_blocks* S, const lif_opts* o, lif_handle* out) {
  g_create_error.clear();
  if (!out || !o) {
    g_create_error = "null argument";
    return LIF_ERR_INVALID;
  }
  *out = nullptr;
  lif_handle h = nullptr;
  try {
    validate_opts(*o);
    check_blocks(S, true, "S");
    LIF_REQUIRE(o->base_rows >= S->b, LIF_ERR_INVALID, "opts.base_rows must be >= b");
    h = new lif_handle_s(o->mem_cap_bytes);
    copy_opts(h, *o);
    Ctx& c = h->ctx;
    c.pool = &h->pool;
    c.b = S->b;
    c.n = S->n;
    c.nb = (int)((S->n + S->b - 1) / S->b);
    Bsr S0 = bsr_from_blocks(c, *S);
    DBuf<double> nrm = block_norms(c, S0);
    h->S = truncate(c, std::move(S0), nrm.get(), h->opts.tau);
    exact_nnzb(c, h->S);
  } catch (const Error& e) {
    g_create_error = e.what();
    delete h;
    return e.status;
  } catch (const std::bad_alloc&) {
    g_create_error = "host allocation failed";
    delete h;
    return LIF_ERR_OUT_OF_MEMORY;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    delete h;
    return LIF_ERR_INVALID;
  }
  *out = h;
  return LIF_OK;
}

lif_status lif_refine(lif_handle h, const lif_blocks* Z0, lif_info* info) {
  if (!h) return LIF_ERR_INVALID;
  return guarded(h, [&] {
    reset_stats(h);
    const auto t0 = std::chrono::steady_clock::now();
    RunInfo ri;
    Bsr Z;
    if (Z0) {
      check_blocks(Z0, false, "Z0");
      LIF_REQUIRE(Z0->n == h->S.n && Z0->b == h->S.b, LIF_ERR_INVALID, "Z0 must have the n and b of S");
      Bsr z = bsr_from_blocks(h->ctx, *Z0);
      Z = run_refine_from(h->ctx, h->S, std::move(z), h->opts, ri);
    } else {
      h->ck.clear();
      h->has_dS = false;
      Z = run_irsi(h->ctx, h->S, h->opts, ri, h->opts.checkpoint ? &h->ck : nullptr);
    }
    h->ctx.sync();
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    h->Z = std::move(Z);
    h->has_Z = true;
    fill_info(h, ri, secs, info);
  });
}

lif_status lif_localized(lif_handle h, lif_info* info) {
  if (!h) return LIF_ERR_INVALID;
  return guarded(h, [&] {
    reset_stats(h);
    const auto t0 = std::chrono::steady_clock::now();
    RunInfo ri;
    h->ck.clear();
    h->has_dS = false;
    Bsr Z = run_lif(h->ctx, h->S, h->opts, ri, h->opts.checkpoint ? &h->ck : nullptr);
    h->ctx.sync();
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    h->Z = std::move(Z);
    h->has_Z = true;
    fill_info(h, ri, secs, info);
  });
}

lif_status lif_rinch(lif_handle h, lif_info* info) {
  if (!h) return LIF_ERR_INVALID;
  return guarded(h, [&] {
    reset_stats(h);
    const auto t0 = std::chrono::steady_clock::now();
    RunInfo ri;
    h->ck.clear();
    h->has_dS = false;
    Bsr Z = run_rinch(h->ctx, h->S, h->opts, ri);
    h->ctx.sync();
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    h->Z = std::move(Z);
    h->has_Z = true;
    fill_info(h, ri, secs, info);
  });
}

lif_status lif_get_Z(lif_handle h, int64_t* nnzb, int32_t* brow, int32_t* bcol, double* vals, int32_t on_device) {
  if (!h) return LIF_ERR_INVALID;
  lif_status st = LIF_OK;
  lif_status g = guarded(h, [&] {
    LIF_REQUIRE(h->has_Z, LIF_ERR_STATE, "no factor yet: call lif_refine or lif_localized first");
    st = copy_out(h, h->Z, nnzb, brow, bcol, vals, on_device);
  });
  return g != LIF_OK ? g : st;
}

lif_status lif_residual(lif_handle h, double* out) {
  if (!h) return LIF_ERR_INVALID;
  return guarded(h, [&] {
    LIF_REQUIRE(out != nullptr, LIF_ERR_INVALID, "out is null");
    LIF_REQUIRE(h->has_Z, LIF_ERR_STATE, "no factor yet: call lif_refine or lif_localized first");
    const Stats keep = h->ctx.stats;
    *out = residual(h->ctx, h->S, h->Z, h->opts.residual_panel_rows);
    h->ctx.flush_timing();
    h->ctx.stats = keep;
  });
}

lif_status lif_residual_against(lif_handle h, const lif_blocks* S, double* out) {
  if (!h) return LIF_ERR_INVALID;
  return guarded(h, [&] {
    LIF_REQUIRE(out != nullptr, LIF_ERR_INVALID, "out is null");
    LIF_REQUIRE(h->has_Z, LIF_ERR_STATE, "no factor yet: call lif_refine or lif_localized first");
    check_blocks(S, false, "S");
    LIF_REQUIRE(S->n == h->S.n && S->b == h->S.b, LIF_ERR_INVALID, "S must have the n and b of the handle");
    const Stats keep = h->ctx.stats;
    double r = 0.0;
    {
      // device blocks are read in place; host blocks are copied once
      Bsr Sx = S->on_device ? bsr_view_blocks(h->ctx, *S) : bsr_from_blocks(h->ctx, *S);
      r = residual(h->ctx, Sx, h->Z, h->opts.residual_panel_rows);
      h->ctx.sync();
    }
    *out = r;
    h->ctx.flush_timing();
    h->ctx.stats = keep;
  });
}

lif_status lif_set_opts(lif_handle h, const lif_opts* o) {
  if (!h) return LIF_ERR_INVALID;
  return guarded(h, [&] {
    LIF_REQUIRE(o != nullptr, LIF_ERR_INVALID, "null options");
    validate_opts(*o);
    LIF_REQUIRE(o->tau == h->opts.tau, LIF_ERR_INVALID,
                "opts.tau cannot change: S was truncated with the handle's threshold");
    LIF_REQUIRE(o->mem_cap_bytes == h->pool.cap(), LIF_ERR_INVALID, "opts.mem_cap_bytes cannot change");
    LIF_REQUIRE(o->base_rows >= h->S.b, LIF_ERR_INVALID, "opts.base_rows must be >= b");
    h->ctx.sync();
    h->ctx.flush_timing();
    copy_opts(h, *o);
    // checkpoints and a kept derivative belong to the previous options' run
    h->ck.clear();
    h->dS = Bsr();
    h->has_dS = false;
  });
}

namespace {

// trunc_tau(alpha op(A) op(B) + gamma D) on the handle, copied out two-phase
lif_status multiply_common(lif_handle h, const lif_blocks* A, int32_t transA, const lif_blocks* B,
                           int32_t transB, double alpha, const lif_blocks* D, double gamma, double tau, int64_t* nnzb,
                           int32_t* brow, int32_t* bcol, double* vals, int32_t on_device, int64_t* products) {
  if (!h) return LIF_ERR_INVALID;
  lif_status st = LIF_OK;
  lif_status g = guarded(h, [&] {
    LIF_REQUIRE(std::isfinite(tau) && tau >= 0.0, LIF_ERR_INVALID, "tau must be finite and >= 0");
    LIF_REQUIRE(std::isfinite(alpha) && std::isfinite(gamma), LIF_ERR_INVALID, "alpha and gamma must be finite");
    check_blocks(A, false, "A");
    check_blocks(B, false, "B");
    LIF_REQUIRE(A->n == h->S.n && A->b == h->S.b && B->n == h->S.n && B->b == h->S.b, LIF_ERR_INVALID,
                "A and B must have the n and b of the handle");
    if (D) {
      check_blocks(D, false, "D");
      LIF_REQUIRE(D->n == h->S.n && D->b == h->S.b, LIF_ERR_INVALID, "D must have the n and b of the handle");
    }
    LIF_REQUIRE((transA & ~(1 | LIF_PRODUCT_UPPER)) == 0 && (transB & ~1) == 0, LIF_ERR_INVALID,
                "transA / transB: unknown flags");
    reset_stats(h);
    Bsr a = bsr_from_blocks(h->ctx, *A);
    Bsr b = bsr_from_blocks(h->ctx, *B);
    Bsr d;
    if (D) d = bsr_from_blocks(h->ctx, *D);
    Bsr C = spgemm(h->ctx, a, (transA & 1) != 0, b, (transB & 1) != 0, tau, h->opts.prec, alpha, D ? &d : nullptr,
                   D ? gamma : 0.0, false, false, (transA & LIF_PRODUCT_UPPER) != 0);
    if (products) *products = h->ctx.stats.products;
    st = copy_out(h, C, nnzb, brow, bcol, vals, on_device);
    h->ctx.sync();
    h->ctx.flush_timing();
  });
  return g != LIF_OK ? g : st;
}

}  // namespace

lif_status lif_multiply(lif_handle h, const lif_blocks* A, int32_t transA, const lif_blocks* B, int32_t transB,
                        double tau, int64_t* nnzb, int32_t* brow, int32_t* bcol, double* vals, int32_t on_device,
                        int64_t* products) {
  return multiply_common(h, A, transA, B, transB, 1.0, nullptr, 0.0, tau, nnzb, brow, bcol, vals, on_device,
                         products);
}

lif_status lif_multiply_add(lif_handle h, const lif_blocks* A, int32_t transA, const lif_blocks* B,
                            int32_t transB, double alpha, const lif_blocks* D, double gamma, double tau,
                            int64_t* nnzb, int32_t* brow, int32_t* bcol, double* vals, int32_t on_device,
                            int64_t* products) {
  return multiply_common(h, A, transA, B, transB, alpha, D, gamma, tau, nnzb, brow, bcol, vals, on_device,
                         products);
}

lif_status lif_backward(lif_handle h, const lif_blocks* G, int64_t* nnzb, int32_t* brow, int32_t* bcol, double* dS,
                        int32_t on_device) {
  if (!h) return LIF_ERR_INVALID;
  lif_status st = LIF_OK;
  lif_status g = guarded(h, [&] {
    LIF_REQUIRE(nnzb != nullptr, LIF_ERR_INVALID, "nnzb is null");
    LIF_REQUIRE(h->ck.valid, LIF_ERR_STATE,
                "no checkpoints: run lif_refine (IRSI) or lif_localized with opts.checkpoint = 1 first");
    if (!h->has_dS || brow == nullptr) {
      check_blocks(G, false, "G");
      LIF_REQUIRE(G->n == h->S.n && G->b == h->S.b, LIF_ERR_INVALID, "G must have the n and b of S");
      Bsr g = bsr_from_blocks(h->ctx, *G);
      h->dS = run_backward(h->ctx, h->S, h->ck, g, h->opts);
      h->has_dS = true;
    }
    st = copy_out(h, h->dS, nnzb, brow, bcol, dS, on_device);
    if (brow != nullptr && st == LIF_OK) {
      h->dS = Bsr();
      h->has_dS = false;
    }
  });
  return g != LIF_OK ? g : st;
}

void lif_destroy(lif_handle h) {
  if (!h) return;
  try {
    h->ctx.sync();
  } catch (...) {
  }
  delete h;
}

const char* lif_last_error(lif_handle h) {
  if (!h) return g_create_error.c_str();
  return h->err.c_str();
}

}  // extern "C"
