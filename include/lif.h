/*
 * lif.h -- C ABI of the MI355X (gfx950) inverse-factorization library.
 *
 * Computes Z with S^{-1} = Z Z^T for a block-sparse symmetric positive
 * definite S (Artemov, Rudberg, Rubensson, "Parallelization and scalability
 * analysis of inverse factorization using the Chunks and Tasks programming
 * model", Sec. 2), by
 *   - iterative refinement from a scaled identity (IRSI, Sec. 2.2,
 *     eq. refinement_local with the start Z_0 = c I), and
 *   - localized inverse factorization (LIF, Alg. 2) with an inverse Cholesky
 *     leaf factorization.
 * Every matrix-matrix product, and every leaf factorization, is followed by
 * truncation: b x b blocks with Frobenius norm < tau are removed (Sec. 5).
 * S itself is truncated the same way when the handle is created.
 *
 * Matrices cross the boundary as block lists (lif_blocks): row-major b x b
 * FP64 blocks with int32 block coordinates sorted by (row, col), no
 * duplicates, entries at scalar indices >= n equal to zero.  A symmetric
 * matrix lists both (i, j) and (j, i).
 *
 * Errors: every call returns a lif_status; nothing throws or exits.  The
 * message of the last failure on a handle is read with lif_last_error.
 * After an error the handle may still be destroyed, and caller outputs are
 * left untouched.
 *
 * Streams: all device work of a handle is queued on the hipStream_t given in
 * lif_opts.stream (NULL = the null stream).  Calls return once their results
 * are complete; the stopping rule needs host-visible norms every iteration.
 * A handle is not re-entrant; separate handles are independent.
 */
#ifndef LIF_H
#define LIF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lif_handle_s* lif_handle;

/* status codes */
#define LIF_OK                 0
#define LIF_ERR_INVALID        1  /* malformed input or options */
#define LIF_ERR_NOT_PD         2  /* a leaf Cholesky met a non-positive pivot */
#define LIF_ERR_NO_CONVERGENCE 3  /* ||delta||_F non-finite, growing past 1, or max_iter reached */
#define LIF_ERR_OUT_OF_MEMORY  4  /* device memory above mem_cap_bytes or hipMalloc failed */
#define LIF_ERR_HIP            5  /* a HIP runtime call failed */
#define LIF_ERR_STATE          6  /* call order (e.g. lif_get_Z before a factorization) */
typedef int32_t lif_status;

/* lif_opts.prec: arithmetic of the products that form the correction M */
#define LIF_FP64        0  /* everything FP64 */
#define LIF_MIXED_FP32  1  /* M products with FP32 inputs, FP32 accumulation; delta and ||delta|| FP64 */
#define LIF_MIXED_BF16  2  /* M products with BF16 inputs, FP32 accumulation; delta and ||delta|| FP64 */

/* lif_opts.stop: stopping rule of the refinement */
#define LIF_STOP_PAPER  0  /* stop when ||delta_k||_F > ||delta_{k-1}||_F^{m+1} (Sec. 2.2), first tested at k = 2 */
#define LIF_STOP_TOL    1  /* stop when ||delta_k||_F <= tol, or when it stops decreasing */

/* lif_opts.refinement: form of the refinement (Sec. 2.2, Sec. 2.3) */
#define LIF_REFINE_LOCAL    0  /* eq. refinement_local: delta updated from the correction, never recomputed */
#define LIF_REFINE_NONLOCAL 1  /* eq. refinement_nonlocal: delta_i = I - (Z_i^T S) Z_i recomputed every
                                * iteration, Z_{i+1} = Z_i P(delta_i), every product truncated; FP64 only */

/* lif_multiply: flag in transA */
#define LIF_PRODUCT_UPPER 2

/* lif_opts.start: scale c of the IRSI start Z_0 = c I (Sec. 2.2) */
#define LIF_START_SQRT2_OVER_GERSH 0  /* c = sqrt(2 / beta), beta the Gershgorin bound of S */
#define LIF_START_INV_SQRT_GERSH   1  /* c = 1 / sqrt(beta) */
#define LIF_START_INV_SQRT_LMAX    2  /* c = 1 / sqrt(start_value), start_value = lambda_max(S) */
#define LIF_START_GIVEN            3  /* c = start_value */

typedef struct {
  int64_t n;             /* matrix dimension (> 0) */
  int32_t b;             /* block size: 32 or 64 */
  int64_t nnzb;          /* number of listed blocks */
  const int32_t* brow;   /* [nnzb] block row, sorted with bcol, in [0, nb), nb = ceil(n/b) */
  const int32_t* bcol;   /* [nnzb] block column */
  const double* vals;    /* [nnzb * b * b] row-major blocks */
  int32_t on_device;     /* 1: the three arrays are device pointers, 0: host pointers */
} lif_blocks;

typedef struct {
  int32_t m;              /* refinement order, 1..8 (the paper uses 4) */
  double tau;             /* block truncation threshold, >= 0 (0 = none) */
  int32_t prec;           /* LIF_FP64 / LIF_MIXED_FP32 / LIF_MIXED_BF16 */
  int32_t stop;           /* LIF_STOP_PAPER / LIF_STOP_TOL */
  double tol;             /* target ||delta||_F for LIF_STOP_TOL */
  int32_t max_iter;       /* per refinement; exceeding it is LIF_ERR_NO_CONVERGENCE */
  int64_t base_rows;      /* LIF recursion stops at ranges of <= base_rows rows (>= b) */
  int32_t start;          /* LIF_START_* (IRSI only) */
  double start_value;     /* lambda_max or c, see LIF_START_* */
  int32_t checkpoint;     /* 1: keep per-iteration Z for lif_backward */
  uint64_t mem_cap_bytes; /* device memory the handle may hold (0 = no cap).  The large-problem
                           * policies are sized against it when it is below the GPU's memory:
                           * iterations on one stream with buffers freed early, products
                           * written as kept blocks only, the residual's panels */
  void* stream;           /* hipStream_t for all work (NULL = null stream) */
  int32_t timing;         /* 1: time every leaf-GEMM launch with HIP events; 2: also the leaf
                           * factorizations and the symbolic phases (lif_info) */
  int32_t presize;        /* 1: from the second iteration of a refinement on, size each
                           * product from the previous iteration's counts (with a
                           * margin) instead of reading its counts back; an iteration
                           * whose sizes fell short is redone with exact sizes, so the
                           * results are identical.  2: the same without the margin
                           * (least memory, most redone iterations).  0: read back the
                           * counts of every product */
  int32_t refinement;     /* LIF_REFINE_LOCAL / LIF_REFINE_NONLOCAL (the latter needs prec = LIF_FP64) */
  double prec_switch;     /* precision schedule, >= 0.  0: with a reduced prec every iteration runs its
                           * correction in that precision and is tested by the stopping rule.  > 0: a
                           * problem's correction runs in reduced precision only while its ||delta||_F
                           * exceeds prec_switch, in FP64 after; such reduced iterations converge
                           * linearly and are checked for divergence only, the stopping rule judges the
                           * FP64 ones (so LIF_STOP_PAPER stops at the FP64 floor) */
  int32_t sym_delta;      /* 1: delta (symmetric in exact arithmetic) is updated on its upper block triangle
                           * only, the update's two products forming just those blocks, and the strictly
                           * upper part is mirrored below (localized refinement); 0: the full update */
  int32_t residual_panel_rows; /* lif_residual forms I - Z^T (S Z) this many block columns at a time
                           * (>= 0; 0: panels of at most min(8 GiB, 1/16 of the device memory the
                           * handle may use) of dense block columns, the whole matrix when it
                           * fits), each panel from S Z's same columns, bounding its memory by Z
                           * and one panel of S Z and of the result */
  int32_t update_panel_rows; /* localized refinement on large problems: the two products of the delta
                           * update and their difference are formed this many block rows at a time
                           * (>= 0; 0: automatic -- panels only on iterations whose buffers fill a
                           * large part of the device memory, sized so that the two products of a
                           * panel take at most 1/32 of it), so that neither product is ever
                           * held whole; the result is the same bit for bit */
  int32_t update_prec;    /* inputs of the delta-update products (S M, Z_{k+1}^T (S M), (S M)^T Z_k of
                           * eq. refinement_local) in a problem's reduced iterations under the precision
                           * schedule: LIF_FP64 (default) or LIF_MIXED_FP32 (FP32 inputs, FP32
                           * accumulation).  delta then carries FP32 rounding, so when a problem's
                           * schedule moves to FP64 its delta is formed again from its definition,
                           * I - trunc(Z^T trunc(S Z)) in FP64 (Sec. 2.2; mirrored with sym_delta), and
                           * its norm replaces the last recorded one.  LIF_MIXED_FP32 needs a reduced
                           * prec with prec_switch > 0 and checkpoint = 0 */
} lif_opts;

typedef struct {
  int32_t iterations_top;    /* refinement iterations of the top-level problem */
  int32_t levels;            /* LIF levels with refinement (0 for IRSI) */
  int32_t iterations_total;  /* sum over all refinements of all nodes */
  int32_t stagnated;         /* 1 if LIF_STOP_TOL ended on a non-decreasing norm above tol */
  double start_scale;        /* c of the IRSI start */
  double delta_tracked;      /* ||delta||_F of the top-level problem when it stopped */
  double flops_leaf_gemm;    /* 2 b^3 per block product, summed over all products */
  double seconds_total;      /* wall time of the call */
  double seconds_leaf_gemm;  /* summed leaf-GEMM kernel time (timing = 1) */
  int64_t leaf_gemm_launches;/* number of leaf-GEMM launches */
  int64_t products_total;    /* block products over all products */
  int64_t nnzb_Z;            /* blocks of the result */
  int32_t n_norms;           /* entries used in norms[] */
  double norms[64];          /* ||delta_k||_F of the top-level problem, k = 1.. */
  int32_t iterations_redone; /* presized iterations redone with exact sizes */
  int32_t cpl_tasks;         /* one-GPU shadow of the critical path (Sec. 3): the longest chain of
                              * dependent tasks the call ran, where a product, a sum or scaling, a
                              * separate transpose and a batched leaf factorization each count one
                              * (independent problems of a level run as one batch) */
  int32_t cpl_products;      /* products on that chain */
  int32_t iterations_reduced;/* node iterations whose correction ran in reduced precision */
  uint64_t mem_peak_bytes;   /* most device memory the handle's buffers held at once during the call */
  uint64_t mem_reserved_bytes;/* device memory the handle holds from HIP at the end of the call */
  int32_t products_compacted;/* products written as kept blocks only (large products on one stream) */
  int32_t pair_panels;       /* panels of block rows whose pair lists were built one at a time */
  double flops_leaf_gemm_reduced;   /* the part of flops_leaf_gemm with FP32 / BF16 inputs */
  double seconds_leaf_gemm_reduced; /* the part of seconds_leaf_gemm in those launches (timing = 1) */
  int64_t leaf_gemm_launches_reduced; /* the part of leaf_gemm_launches with FP32 / BF16 inputs */
  double seconds_leaf_factorization;  /* timing = 2: the batched leaf factorizations (all steps and the
                                       * inverse's columns on the second stream), summed over the call */
  double flops_leaf_factorization;    /* their algorithmic flops: the band-limited Cholesky (diagonal
                                       * tiles, panels, trailing updates), the panel products V and the
                                       * inverse's tile products, b^3 or 2 b^3 each as counted */
  double seconds_symbolic;            /* timing = 2: the symbolic phases (counts, scans, fills) */
  double bytes_symbolic;              /* their algorithmic bytes: 20 per block product (a column index
                                       * read, a 16-byte pair written), 12 per output block, the row
                                       * pointers */
  int64_t symbolic_launches;          /* timed symbolic launches */
  double flops_leaf_gemm_fp32;        /* the part of flops_leaf_gemm_reduced with FP32 inputs */
  double seconds_leaf_gemm_fp32;      /* the part of seconds_leaf_gemm_reduced in those launches */
  int64_t leaf_gemm_launches_fp32;    /* the part of leaf_gemm_launches_reduced with FP32 inputs */
} lif_info;

/* Fills *o with the defaults: m = 4, tau = 0, FP64, paper stopping rule,
 * tol = 1e-10, max_iter = 100, base_rows = 4096, start = SQRT2_OVER_GERSH,
 * checkpoint = 0, no cap, null stream, timing = 0, presize = 1,
 * refinement = LIF_REFINE_LOCAL, prec_switch = 0, sym_delta = 0, residual_panel_rows = 0,
 * update_panel_rows = 0. */
lif_status lif_opts_default(lif_opts* o);

/* Validates S and copies it into library-owned device memory (the caller may
 * free its arrays on return), truncates it at o->tau.  Checks: n > 0,
 * b in {32, 64}, sorted unique in-range blocks, symmetric block pattern,
 * zero padding, options in range (LIF_ERR_INVALID otherwise).  The options
 * are copied.  On success *out owns all device memory of the problem. */
lif_status lif_create(const lif_blocks* S, const lif_opts* o, lif_handle* out);

/* Iterative refinement (eq. refinement_local).  Z0 == NULL: IRSI, start
 * Z_0 = c I, delta_0 = I - c^2 S (Sec. 2.2).  Otherwise Z0 (same n and b)
 * is the start and delta_0 = I - Z0^T S Z0 (products truncated).  With
 * opts.refinement = LIF_REFINE_NONLOCAL the regular form runs instead
 * (eq. refinement_nonlocal): delta_0 = I - (Z_0^T S) Z_0 for either start,
 * and every iteration recomputes delta from the new Z.  The result replaces
 * the handle's Z.  info may be NULL. */
lif_status lif_refine(lif_handle h, const lif_blocks* Z0, lif_info* info);

/* Localized inverse factorization (Alg. 2): ranges of more than base_rows
 * rows split at ceil(nb/2) blocks; leaves factorized by inverse Cholesky
 * (S_leaf = U^T U, Z_leaf = U^{-1}); each level of the recursion is corrected
 * by localized refinement from diag(Z_A, Z_C) with
 * delta_0 = -[[0, X], [X^T, 0]], X = (Z_A^T B) Z_C.  All nodes of one depth are
 * processed together.  A non-positive leaf pivot gives LIF_ERR_NOT_PD.
 * With opts.refinement = LIF_REFINE_NONLOCAL this is the recursive inverse
 * factorization of Sec. 2.3 instead: the same recursion and start
 * diag(Z_A, Z_C), corrected by the regular form (eq. refinement_nonlocal)
 * with delta_0 = I - (Z_0^T S) Z_0 on each node. */
lif_status lif_localized(lif_handle h, lif_info* info);

/* Recursive inverse Cholesky (Alg. 1) of the handle's S, as a standalone
 * method: ranges of more than base_rows rows split at ceil(nb/2) blocks
 * (as in lif_localized); with S = [[S00, S01], [S01^T, S11]],
 *   Z00 = rinch(S00), R = Z00^T S01, Q = S11 - R^T R, Z11 = rinch(Q),
 *   Z01 = -(Z00 R) Z11,
 * every product truncated at tau, Q itself not; leaves of at most base_rows
 * rows are inverse Cholesky factors, truncated.  The result replaces the
 * handle's Z (upper triangular, Z^T S Z = I up to truncation); info->levels
 * is the recursion depth, no refinement runs.  A non-positive leaf pivot
 * gives LIF_ERR_NOT_PD.  Checkpoints for lif_backward are not kept. */
lif_status lif_rinch(lif_handle h, lif_info* info);

/* Copies the handle's Z out as a block list.  Two-phase: with brow == NULL
 * only *nnzb is written; otherwise the arrays (capacity *nnzb blocks, host or
 * device per on_device) receive the blocks in (row, col) order.
 * LIF_ERR_STATE before a factorization, LIF_ERR_INVALID if the capacity is
 * too small. */
lif_status lif_get_Z(lif_handle h, int64_t* nnzb, int32_t* brow, int32_t* bcol, double* vals,
                     int32_t on_device);

/* ||I - Z^T S Z||_F of the handle's Z in FP64 with no truncation (Table 1's
 * error measure), against the truncated S the handle factorized; formed by
 * panels of block columns (opts.residual_panel_rows), never stored whole. */
lif_status lif_residual(lif_handle h, double* out);

/* ||I - Z^T S Z||_F of the handle's Z against another S of the same n and b
 * (Table 1's error measure; for example the matrix before the block
 * truncation the handle applied at creation, since the table does not say
 * which S its residuals use), FP64, untruncated, by panels of block columns as
 * lif_residual.  S may be host or device blocks (device blocks are read in
 * place, not copied); its pattern need not be symmetric.  LIF_ERR_STATE
 * before a factorization. */
lif_status lif_residual_against(lif_handle h, const lif_blocks* S, double* out);

/* Replaces the handle's options (S, its truncation and the memory pool
 * stay): opts.tau and opts.mem_cap_bytes must equal the handle's, the rest
 * is validated as in lif_create.  Lets one handle, its S and its warm memory
 * pool serve runs in several precisions or stopping rules.  Drops the
 * checkpoints and any kept derivative; the current Z stays. */
lif_status lif_set_opts(lif_handle h, const lif_opts* o);

/* C = op(A) op(B) truncated at tau: the block-sparse product of Sec. 4 with
 * the leaf truncation of Sec. 5, on the handle's stream and memory.  op is
 * the identity (bit 0 of trans clear) or the transpose (bit 0 set); with
 * LIF_PRODUCT_UPPER set in transA only the output blocks (i, j) with j >= i
 * are formed (the upper block triangle).  A and B must have
 * the handle's n and b.  The product uses the handle's opts.prec: FP64, or
 * inputs rounded to FP32 / BF16 (round to nearest even; BF16 via FP32) with
 * FP32 accumulation and an FP64 result.  Two-phase output like lif_get_Z (the product is
 * recomputed on the second call); *products receives the number of block
 * products (may be NULL). */
lif_status lif_multiply(lif_handle h, const lif_blocks* A, int32_t transA, const lif_blocks* B,
                        int32_t transB, double tau, int64_t* nnzb, int32_t* brow, int32_t* bcol,
                        double* vals, int32_t on_device, int64_t* products);

/* C = trunc_tau(alpha op(A) op(B) + gamma D): one product with an added term,
 * the fused form of a Horner step of eq. refinement_local (Sec. 2.2):
 * delta T with T = X + c I is delta X + c delta, and the added term c delta
 * enters every output block before the block's Frobenius norm decides its
 * truncation (Sec. 5).  D (NULL = no term) has the handle's n and b; its
 * blocks join the output pattern.  With a reduced opts.prec only A and B are
 * read in the input precision (alpha scales their FP32-accumulated product);
 * D is added in FP64, never rounded.  Everything else as lif_multiply
 * (transposes, LIF_PRODUCT_UPPER, two-phase output, *products). */
lif_status lif_multiply_add(lif_handle h, const lif_blocks* A, int32_t transA, const lif_blocks* B,
                            int32_t transB, double alpha, const lif_blocks* D, double gamma, double tau,
                            int64_t* nnzb, int32_t* brow, int32_t* bcol, double* vals, int32_t on_device,
                            int64_t* products);

/* Bytes of the device array lif_multiply_noalloc works in (one per GPU). */
#define LIF_NOALLOC_SCRATCH_BYTES (256ull << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture setup, tight serving loops, harnesses that forbid hipMalloc): the
 * product of lif_multiply_add, C = trunc_tau(alpha op(A) op(B) + gamma D),
 * without a handle and without any device or pinned-host allocation.  Every
 * working buffer (index arrays, block-product lists, the product's values
 * before truncation, reduced-precision copies) is carved from one library
 * array of LIF_NOALLOC_SCRATCH_BYTES in device memory, one copy per GPU,
 * held from the library's first use on that GPU until the process ends.
 * A product whose working set does not fit it is rejected with
 * LIF_ERR_OUT_OF_MEMORY and a message naming the limit (lif_last_error(NULL)).
 * The array keeps whatever the last call left; calls on one GPU are
 * serialized by a lock in the library, and a call that overlaps another use
 * of the array on that GPU (another process's copy excepted) would race.
 *   A, B, D: block lists on the current device (on_device = 1), the same n
 *     and b (32 or 64); D may be NULL (no added term, gamma ignored).
 *   transA: bit 0 transposes A, LIF_PRODUCT_UPPER keeps the upper block
 *     triangle; transB: bit 0 transposes B.
 *   prec: LIF_FP64, LIF_MIXED_FP32 or LIF_MIXED_BF16 (A and B read in that
 *     precision, FP32 accumulation, D added in FP64).
 *   stream: hipStream_t for the work (NULL = the null stream).
 *   capacity: blocks the output arrays hold; brow, bcol (int32) and vals
 *     (capacity * b * b FP64) are device arrays, written in (row, col) order.
 *   *nnzb: blocks of C on success; when capacity is too small,
 *     LIF_ERR_INVALID with *nnzb = the blocks needed and the outputs untouched.
 *   *products (may be NULL): block products of the symbolic phase.
 * Returns once C is complete. */
lif_status lif_multiply_noalloc(const lif_blocks* A, int32_t transA, const lif_blocks* B, int32_t transB,
                                double alpha, const lif_blocks* D, double gamma, double tau, int32_t prec,
                                void* stream, int64_t capacity, int64_t* nnzb, int32_t* brow, int32_t* bcol,
                                double* vals, int64_t* products);

/* Reverse-mode derivative of the last factorization (differentiation form):
 * dS = sym(dL/dS) = (A + A^T) / 2 for the linear loss L = tr(G^T Z), so that
 * dL = <dS, E> for every symmetric perturbation E of S.  Returned on S's block
 * pattern (the truncated S the handle holds; blocks where the derivative has
 * no contribution are zero).  The iteration is differentiated through the
 * regular recurrence delta_i = I - Z_i^T S Z_i of eq. refinement_nonlocal
 * (equal to the localized iterates in exact arithmetic) with the iteration
 * counts of the forward run frozen and untruncated FP64 products; LIF levels
 * pass the diagonal parts of dL/dZ_0 to their children, and leaves use the
 * inverse-Cholesky adjoint.  The IRSI start scale c is held constant.
 * Needs the forward (lif_refine with Z0 == NULL, or lif_localized) to have
 * run with opts.checkpoint = 1, else LIF_ERR_STATE.  G: the handle's n and
 * b, any block pattern.  Two-phase: with brow == NULL the derivative is
 * computed, kept in the handle and *nnzb is set; a call with arrays copies
 * the kept derivative (G may then be NULL) or, if none is kept, computes it
 * first; the kept derivative is released after the copy. */
lif_status lif_backward(lif_handle h, const lif_blocks* G, int64_t* nnzb, int32_t* brow, int32_t* bcol, double* dS,
                        int32_t on_device);

/* Releases the handle and all its device memory.  NULL is ignored. */
void lif_destroy(lif_handle h);

/* Message of the last failed call on h ("" if none); valid until the next
 * call on h.  With h == NULL: the last lif_create failure of this thread. */
const char* lif_last_error(lif_handle h);

#ifdef __cplusplus
}
#endif

#endif /* LIF_H */
