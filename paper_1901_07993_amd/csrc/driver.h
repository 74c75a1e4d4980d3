// Drivers of the three refinement-based computations: IRSI (Sec. 2.2),
// localized inverse factorization (Alg. 2) with a batched inverse Cholesky
// leaf, and the untruncated residual ||I - Z^T S Z||_F (Table 1).
#pragma once

#include "common.h"

namespace lif {

struct Opts {
  int m = 4;
  double tau = 0.0;
  int prec = LIF_FP64;
  int stop = LIF_STOP_PAPER;
  double tol = 1e-10;
  int max_iter = 100;
  int64_t base_rows = 4096;
  int start = LIF_START_SQRT2_OVER_GERSH;
  double start_value = 0.0;
  bool checkpoint = false;
  int presize = 1;  // 0 off, 1 with margins, 2 previous counts as they are
  int refinement = LIF_REFINE_LOCAL;
  double prec_switch = 0.0;  // > 0: reduced precision only while ||delta||_F exceeds it
  bool sym_delta = false;    // update delta's upper block triangle and mirror it
  int residual_panel_rows = 0;  // block rows of I - Z^T S Z formed at once (0: automatic)
  int update_panel_rows = 0;    // block rows of the delta update formed at once (0: automatic)
  int update_prec = 0;          // inputs of the delta update in reduced iterations (LIF_FP64 / LIF_MIXED_FP32)
};

// One node of the split tree: scalar rows [lo, hi), lo a multiple of b.
struct PlanNode {
  int64_t lo, hi;
  int depth;
  int left = -1, right = -1;  // children (indices into the plan), -1 for a leaf
};

struct Plan {
  std::vector<PlanNode> nodes;  // nodes[0] is the root
  int max_depth = 0;
};

// Split rule: a range of more than base_rows rows is split after its
// ceil(nb/2) leading blocks.
Plan make_plan(int64_t n, int b, int64_t base_rows);

struct RunInfo {
  int iterations_top = 0;
  int levels = 0;
  int iterations_total = 0;
  bool stagnated = false;
  double start_scale = 0.0;
  double delta_top = 0.0;
  std::vector<double> norms_top;
  int iterations_reduced = 0;  // node iterations with a reduced-precision correction
};

// Per-iteration checkpoints of a forward run, for the reverse sweep.
// A level is one batch of independent problems refined together (IRSI: one
// problem on all rows).
struct LevelCk {
  std::vector<int> rlo, rhi;   // block-row range of each problem
  std::vector<int> iters;      // refinement iterations of each problem
  std::vector<Bsr> Z;          // Z before each batch iteration: Z_0 .. Z_{K-1}
  Bsr S_lvl;                   // the level's block-diagonal S (empty: the handle's S)
  std::vector<int> part_lab;   // per block row: the part (child) the row belongs to after the split
};

struct Checkpoints {
  bool valid = false;
  bool lif = false;
  std::vector<LevelCk> levels;  // top level first
  Bsr Z_leaf;                   // LIF: the leaf factors (block diagonal, upper triangular)
  void clear() {
    valid = lif = false;
    levels.clear();
    Z_leaf = Bsr();
  }
};

// Identity-like helpers on the context: a per-block-row flag array with
// every row set.
const unsigned char* all_rows_on(Ctx& c);

// IRSI: Z_0 = c I, delta_0 = I - c^2 S.  ck (may be null) receives the
// per-iteration checkpoints.
Bsr run_irsi(Ctx& c, const Bsr& S, const Opts& o, RunInfo& info, Checkpoints* ck = nullptr);
// Refinement from a given start: delta_0 = I - Z0^T S Z0 (products truncated).
Bsr run_refine_from(Ctx& c, const Bsr& S, Bsr&& Z0, const Opts& o, RunInfo& info);
// Localized inverse factorization.
Bsr run_lif(Ctx& c, const Bsr& S, const Opts& o, RunInfo& info, Checkpoints* ck = nullptr);
// Recursive inverse Cholesky (Alg. 1), split like LIF; info.levels = the
// recursion depth (leaves included).
Bsr run_rinch(Ctx& c, const Bsr& S, const Opts& o, RunInfo& info);
// Reverse sweep: sym(dL/dS) on S's block pattern for L = tr(G^T Z), through
// the regular recurrence delta_i = I - Z_i^T S Z_i with the checkpointed Z_i
// and frozen iteration counts; untruncated FP64 products.
Bsr run_backward(Ctx& c, const Bsr& S, const Checkpoints& ck, const Bsr& G, const Opts& o);
// Batched leaf factorization of the diagonal ranges [lo_k, hi_k) of S:
// block-diagonal upper-triangular Z with Z_k^T S_k Z_k = I, truncated at tau.
Bsr leaf_inverse_cholesky(Ctx& c, const Bsr& S, const std::vector<std::pair<int64_t, int64_t>>& ranges,
                          double tau);
// ||I - Z^T S Z||_F with untruncated products, formed `panel_rows` block rows
// at a time (0: panels of at most 8 GiB of dense block rows).
double residual(Ctx& c, const Bsr& S, const Bsr& Z, int panel_rows = 0);

}  // namespace lif
