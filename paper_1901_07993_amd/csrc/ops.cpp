// Block-sparse operations on device block-CSR matrices.  Each operation
// allocates its outputs from the handle's pool and queues its kernels on the
// handle's stream.  Only the symbolic phase of a product reads sizes back to
// the host (it has no host-known bound), and not even that when the caller
// planned its capacities (Ctx::Spec); truncation, filters and sums size
// their outputs by a bound and leave the exact count on the device.
#include <algorithm>

#include <cstdio>

#include "common.h"

namespace lif {

namespace {

template <typename T>
T read1(Ctx& c, const T* dev) {
  T v;
  c.d2h(&v, dev, sizeof(T));
  return v;
}

// operations that read every stored block take no matrix with holes
void no_holes(const Bsr& A, const char* op) {
  LIF_REQUIRE(!A.holes, LIF_ERR_INVALID, std::string(op) + ": operand with dropped blocks not compacted");
}

Bsr like(const Bsr& A) {
  Bsr C;
  C.n = A.n;
  C.b = A.b;
  C.nb = A.nb;
  C.cpl = A.cpl;
  C.cpl_products = A.cpl_products;
  return C;
}

}  // namespace

void task_after(Ctx& c, Bsr& out, bool product, std::initializer_list<const Bsr*> in) {
  int d = 0, p = 0;
  for (const Bsr* x : in)
    if (x && (x->cpl > d || (x->cpl == d && x->cpl_products > p))) {
      d = x->cpl;
      p = x->cpl_products;
    }
  out.cpl = d + 1;
  out.cpl_products = p + (product ? 1 : 0);
  if (out.cpl > c.stats.cpl || (out.cpl == c.stats.cpl && out.cpl_products > c.stats.cpl_products)) {
    c.stats.cpl = out.cpl;
    c.stats.cpl_products = out.cpl_products;
  }
}

bool exact_store_pays(Ctx& c, int64_t blocks, int b) {
  const double bytes = (double)blocks * b * b * sizeof(double);
  return bytes > std::min(double(1u << 30), (double)c.device_bytes() / 64.0);
}

Store new_store(Ctx& c, int64_t blocks, int b) {
  return std::make_shared<DBuf<double>>(c.pool, (size_t)std::max<int64_t>(blocks, 0) * b * b);
}

Bsr compact_values(Ctx& c, Bsr&& A) {
  no_holes(A, "compact_values");
  const int64_t nnz = exact_nnzb(c, A);
  Store st = new_store(c, nnz, A.b);
  launch_gather_values(c, A.ptrs(), nnz, A.b, st->get(), nullptr);
  launch_fill_ptrs(c, A.blk.get(), st->get(), A.b, nnz);
  A.store.assign(1, st);
  A.lp[0] = Bsr::Shadow();  // the copies point at the old blocks' places
  A.lp[1] = Bsr::Shadow();
  return std::move(A);
}

void ensure_shadow(Ctx& c, const Bsr& A, int prec, int layout) {
  Bsr::Shadow& s = A.lp[layout];
  if (s.prec == prec) return;
  s = Bsr::Shadow();
  const int64_t n = A.bound();
  const size_t bytes = (size_t)n * A.b * A.b * (prec == LIF_MIXED_BF16 ? 2 : 4);
  s.store = std::make_shared<DBuf<double>>(c.pool, (bytes + 7) / 8);
  s.ptr = DBuf<const void*>(c.pool, (size_t)n);
  launch_make_shadow(c, prec, layout == 1, A.ptrs(), n, A.live(), A.b, s.store->get(), s.ptr.get());
  s.prec = prec;
}

int64_t exact_nnzb(Ctx& c, const Bsr& A) {
  if (A.nnzb < 0) A.nnzb = read1(c, A.live());
  return A.nnzb;
}

Bsr bsr_empty(Ctx& c, int64_t n, int b) {
  Bsr A;
  A.n = n;
  A.b = b;
  A.nb = (int)((n + b - 1) / b);
  A.nnzb = 0;
  A.cap = 0;
  A.row_ptr = DBuf<int>(c.pool, A.nb + 1);
  launch_fill_i32(c, A.row_ptr.get(), 0, A.nb + 1);
  return A;
}

Bsr bsr_from_blocks(Ctx& c, const lif_blocks& in) {
  Bsr A;
  A.n = in.n;
  A.b = in.b;
  A.nb = (int)((in.n + in.b - 1) / in.b);
  A.nnzb = in.nnzb;
  A.cap = in.nnzb;
  const hipMemcpyKind kind = in.on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  DBuf<int> brow(c.pool, (size_t)in.nnzb);
  A.col = DBuf<int>(c.pool, (size_t)in.nnzb);
  Store st = new_store(c, in.nnzb, in.b);
  A.blk = DBuf<const double*>(c.pool, (size_t)in.nnzb);
  A.store.push_back(st);
  if (in.nnzb) {
    LIF_HIP(hipMemcpyAsync(brow.get(), in.brow, in.nnzb * sizeof(int), kind, c.stream));
    LIF_HIP(hipMemcpyAsync(A.col.get(), in.bcol, in.nnzb * sizeof(int), kind, c.stream));
    LIF_HIP(hipMemcpyAsync(st->get(), in.vals, in.nnzb * (size_t)in.b * in.b * sizeof(double), kind, c.stream));
    launch_fill_ptrs(c, A.blk.get(), st->get(), in.b, in.nnzb);
  }
  A.row_ptr = DBuf<int>(c.pool, A.nb + 1);
  launch_row_ptr_from_rows(c, brow.get(), in.nnzb, A.nb, A.row_ptr.get());
  return A;
}

Bsr bsr_view_blocks(Ctx& c, const lif_blocks& in) {
  LIF_REQUIRE(in.on_device, LIF_ERR_INVALID, "bsr_view_blocks: the block list must be on the device");
  Bsr A;
  A.n = in.n;
  A.b = in.b;
  A.nb = (int)((in.n + in.b - 1) / in.b);
  A.nnzb = in.nnzb;
  A.cap = in.nnzb;
  A.col = DBuf<int>(c.pool, (size_t)in.nnzb);
  A.blk = DBuf<const double*>(c.pool, (size_t)in.nnzb);
  if (in.nnzb) {
    LIF_HIP(hipMemcpyAsync(A.col.get(), in.bcol, in.nnzb * sizeof(int), hipMemcpyDeviceToDevice, c.stream));
    // the caller's blocks are only read: the block pointers address them in place
    launch_fill_ptrs(c, A.blk.get(), in.vals, in.b, in.nnzb);
  }
  A.row_ptr = DBuf<int>(c.pool, A.nb + 1);
  launch_row_ptr_from_rows(c, in.brow, in.nnzb, A.nb, A.row_ptr.get());
  return A;
}

void bsr_to_blocks(Ctx& c, const Bsr& A, int32_t* brow, int32_t* bcol, double* vals, bool on_device) {
  no_holes(A, "bsr_to_blocks");
  const int64_t nnz = exact_nnzb(c, A);
  if (nnz == 0) return;
  DBuf<int> rows(c.pool, (size_t)nnz);
  launch_block_row_of(c, A.row_ptr.get(), A.nb, nnz, rows.get());
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  LIF_HIP(hipMemcpyAsync(brow, rows.get(), nnz * sizeof(int), kind, c.stream));
  LIF_HIP(hipMemcpyAsync(bcol, A.col.get(), nnz * sizeof(int), kind, c.stream));
  if (on_device) {
    launch_gather_values(c, A.ptrs(), nnz, A.b, vals, nullptr);
  } else {
    DBuf<double> tmp(c.pool, (size_t)nnz * A.b * A.b);
    launch_gather_values(c, A.ptrs(), nnz, A.b, tmp.get(), nullptr);
    LIF_HIP(hipMemcpyAsync(vals, tmp.get(), nnz * (size_t)A.b * A.b * sizeof(double), kind, c.stream));
    c.sync();
  }
  c.sync();
}

Bsr copy(Ctx& c, const Bsr& A) {
  Bsr B = like(A);
  B.nnzb = A.nnzb;
  B.cap = A.bound();
  B.row_ptr = DBuf<int>(c.pool, A.nb + 1);
  B.col = DBuf<int>(c.pool, (size_t)B.cap);
  B.blk = DBuf<const double*>(c.pool, (size_t)B.cap);
  B.holes = A.holes;
  B.share_store(A);  // the value blocks are shared, never written again
  LIF_HIP(hipMemcpyAsync(B.row_ptr.get(), A.row_ptr.get(), (A.nb + 1) * sizeof(int), hipMemcpyDeviceToDevice,
                         c.stream));
  if (B.cap) {
    LIF_HIP(hipMemcpyAsync(B.col.get(), A.col.get(), B.cap * sizeof(int), hipMemcpyDeviceToDevice, c.stream));
    LIF_HIP(hipMemcpyAsync(B.blk.get(), A.blk.get(), B.cap * sizeof(const double*), hipMemcpyDeviceToDevice,
                           c.stream));
  }
  return B;
}

DBuf<double> block_norms(Ctx& c, const Bsr& A) {
  no_holes(A, "block_norms");
  DBuf<double> nrm(c.pool, (size_t)A.bound());
  launch_block_sumsq(c, A.ptrs(), A.bound(), A.b, nrm.get(), true, A.live());
  return nrm;
}

// Sec. 5 truncation: drop blocks with Frobenius norm < tau, keep the order.
// The kept count stays on the device; the capacity is the input's bound.
Bsr truncate(Ctx& c, Bsr&& A, const double* norms, double tau) {
  no_holes(A, "truncate");
  if (tau <= 0.0 || A.bound() == 0) return std::move(A);
  Bsr B = like(A);
  B.nnzb = -1;
  B.cap = A.bound();
  B.row_ptr = DBuf<int>(c.pool, A.nb + 1);
  launch_keep_count_scan(c, A.row_ptr.get(), norms, tau, A.nb, B.row_ptr.get());
  B.col = DBuf<int>(c.pool, (size_t)B.cap);
  B.blk = DBuf<const double*>(c.pool, (size_t)B.cap);
  B.share_store(A);
  launch_compact_gather(c, A.row_ptr.get(), A.nb, A.col.get(), norms, tau, B.row_ptr.get(), A.ptrs(), A.bound(),
                        B.col.get(), B.blk.get());
  return B;
}

CsrView transpose_view(Ctx& c, const Bsr& A) {
  CsrView v;
  const int nb = A.nb;
  const int64_t cap = A.bound();
  DBuf<int> cnt(c.pool, nb);
  v.own_rp = DBuf<int>(c.pool, nb + 1);
  if (transpose_count_scan_fits(nb)) {  // counts, scan and cleared cursors in one launch
    launch_transpose_count_scan(c, A.col.get(), cap, A.live(), nb, v.own_rp.get(), cnt.get());
  } else {
    launch_fill_i32(c, cnt.get(), 0, nb);
    launch_transpose_counts(c, A.col.get(), cap, cnt.get(), A.live());
    scan_exclusive_i32(c, cnt.get(), v.own_rp.get(), nb);
    launch_fill_i32(c, cnt.get(), 0, nb);
  }
  DBuf<int> tcol(c.pool, (size_t)cap), tsrc(c.pool, (size_t)cap);
  if (cap)
    launch_transpose_fill(c, A.row_ptr.get(), A.col.get(), v.own_rp.get(), nb, cnt.get(), tcol.get(), tsrc.get());
  v.own_col = DBuf<int>(c.pool, (size_t)cap);
  v.own_idx = DBuf<int>(c.pool, (size_t)cap);
  if (cap) launch_transpose_sort(c, v.own_rp.get(), nb, tcol.get(), tsrc.get(), v.own_col.get(), v.own_idx.get());
  v.rp = v.own_rp.get();
  v.col = v.own_col.get();
  v.idx = v.own_idx.get();
  return v;
}

Bsr transpose(Ctx& c, const Bsr& A) {
  no_holes(A, "transpose");
  // a large matrix known only by a bound (a filter of a sum) gets its exact
  // count first: the transposed values are stored for that many blocks
  if (A.nnzb < 0 && exact_store_pays(c, A.bound(), A.b)) exact_nnzb(c, A);
  CsrView v = transpose_view(c, A);
  Bsr T = like(A);
  T.nnzb = A.nnzb;
  T.cap = A.bound();
  T.row_ptr = std::move(v.own_rp);
  T.col = std::move(v.own_col);
  Store st = new_store(c, T.cap, A.b);
  T.blk = DBuf<const double*>(c.pool, (size_t)T.cap);
  T.store.push_back(st);
  launch_transpose_blocks(c, A.ptrs(), v.own_idx.get(), T.cap, A.b, st->get(), T.blk.get(), T.live());
  task_after(c, T, false, {&A});  // a separate transpose is a task
  return T;
}

namespace {

// Output stores above min(512 MiB, 1/64 of the device memory the handle may
// use) are written compacted (kept blocks only), in chunks of at most
// min(4 GiB, 1/16 of it) of untruncated output; pair lists above
// min(2 GiB, 1/512 of it) are built one panel of block rows at a time when
// the product is compacted and memory is short (the list above 1/64 of it,
// or taking the pool past half of it): each panel ends in a drain of the
// GPU, a cost paid only there.
constexpr double kCompactMinBytes = 512.0 * double(1u << 20);
constexpr double kCompactChunkBytes = 4.0 * double(1u << 30);
constexpr double kPairPanelBytes = 2.0 * double(1u << 30);

// Whether a product of `blocks` output blocks is written compacted: only
// where freed memory is reusable at once (one stream); with a memory cap
// whenever the store is large, without one only when memory is short (the
// untruncated store would take the buffers in use past half of the GPU's
// memory): the chunks' read-backs and slot atomics cost about 6 % of the
// products' time on a water cluster that fits without them.
bool compact_output(Ctx& c, int64_t blocks, int b) {
  const double dev = (double)c.device_bytes(), bytes = (double)blocks * b * b * sizeof(double);
  return !c.pool->deferring() && bytes > std::min(kCompactMinBytes, dev / 64.0) &&
         (c.pool->cap() != 0 || (double)c.pool->in_use() + bytes > 0.5 * dev);
}

// Numeric phase of output blocks [e0, e1) of C (pattern and blk array
// allocated), compacted: kept blocks only, written to consecutive slots of
// one store per chunk of output blocks, each store cut to its kept blocks
// once the chunk is done (a read-back per chunk), so that the untruncated
// product is never held.  Dropped blocks get null pointers.  A
// reduced-precision copy for the next product is made by that product.
void numeric_compacted(Ctx& c, Bsr& C, int prec, bool ta, bool tb, const int64_t* seg, const BlockPair* pairs,
                       int64_t e0, int64_t e1, const Epilogue& epi) {
  const double blk_bytes = (double)C.b * C.b * sizeof(double);
  const double dev = (double)c.device_bytes();
  const int64_t chunk = std::max<int64_t>(1, (int64_t)(std::min(kCompactChunkBytes, dev / 16.0) / blk_bytes));
  DBuf<unsigned long long> kept(c.pool, 1);
  if (e0 == 0) ++c.stats.compacted;  // counted once per product
  for (int64_t a = e0; a < e1; a += chunk) {
    const int64_t n = std::min(chunk, e1 - a);
    Store st = new_store(c, n, C.b);
    launch_fill_i32(c, reinterpret_cast<int*>(kept.get()), 0, 2);
    Epilogue e = epi;
    e.slots = kept.get();
    e.dsrc = epi.dsrc ? epi.dsrc + a : nullptr;
    launch_numeric(c, prec, ta, tb, seg + a, pairs, n, nullptr, C.b, st->get(), C.blk.get() + a, nullptr, e);
    unsigned long long k = 0;
    c.d2h_batch({{&k, kept.get(), sizeof(k)}});
    st->shrink((size_t)k * C.b * C.b);
    if (k) C.store.push_back(st);
  }
}

// The numeric phase of a product whose pattern, segments and pairs are
// built: values, norms, truncation (or holes).
// `poison` (nullable): the flag that voids the product (Epilogue).
Bsr numeric_phase(Ctx& c, Bsr&& C, bool ta, bool tb, double tau, int prec, double alpha, BlkIn dsrc, double gamma,
                  bool keep_holes, const int64_t* seg, const BlockPair* pairs, int64_t nnzc, const int* poison,
                  bool out_lp) {
  const int nb = C.nb;
  C.blk = DBuf<const double*>(c.pool, (size_t)nnzc);
  Epilogue epi;
  epi.alpha = alpha;
  epi.gamma = gamma;
  epi.dsrc = dsrc;
  epi.poison = poison;
  epi.rows = C.row_ptr.get();
  epi.nrows = nb;
  const double blk_bytes = (double)C.b * C.b * sizeof(double);
  const double dev = (double)c.device_bytes();
  if (keep_holes && tau > 0.0 && !poison && compact_output(c, nnzc, C.b)) {
    epi.drop = true;
    epi.tau = tau;
    C.holes = true;
    numeric_compacted(c, C, prec, ta, tb, seg, pairs, 0, nnzc, epi);
    return std::move(C);
  }
  Store st = new_store(c, nnzc, C.b);
  C.store.push_back(st);
  if (out_lp && keep_holes && prec != LIF_FP64 && nnzc > 0) {
    // the result's transposed input-precision copy, written with its blocks
    Bsr::Shadow& sh = C.lp[1];
    const size_t bytes = (size_t)nnzc * C.b * C.b * (prec == LIF_MIXED_BF16 ? 2 : 4);
    sh.store = std::make_shared<DBuf<double>>(c.pool, (bytes + 7) / 8);
    sh.ptr = DBuf<const void*>(c.pool, (size_t)nnzc);
    sh.prec = prec;
    epi.lp_store = sh.store->get();
    epi.lp_ptr = sh.ptr.get();
  }
  if (keep_holes && tau > 0.0) {  // truncation by null pointers, no compaction
    epi.drop = true;
    epi.tau = tau;
    C.holes = true;
    launch_numeric(c, prec, ta, tb, seg, pairs, nnzc, C.row_ptr.get() + nb, C.b, st->get(), C.blk.get(), nullptr,
                   epi);
    return std::move(C);
  }
  DBuf<double> nrm(c.pool, (size_t)nnzc);
  launch_numeric(c, prec, ta, tb, seg, pairs, nnzc, C.row_ptr.get() + nb, C.b, st->get(), C.blk.get(), nrm.get(),
                 epi);
  return truncate(c, std::move(C), nrm.get(), tau);
}

}  // namespace

namespace {

Bsr spgemm_body(Ctx& c, const Bsr& A, bool ta, const Bsr& B, bool tb, double tau, int prec, double alpha,
                const Bsr* D, double gamma, bool keep_holes, bool out_lp, bool upper) {
  LIF_REQUIRE(A.nb == B.nb && A.b == B.b, LIF_ERR_INVALID, "spgemm: operand shapes differ");
  // block pointers the pairs are built from: the FP64 blocks, or for a
  // reduced-precision product op(A)'s blocks row-major and op(B)'s blocks
  // transposed in the input precision
  BlkIn pa = A.ptrs(), pb = B.ptrs();
  if (prec != LIF_FP64) {
    const int la = ta ? 1 : 0, lb = tb ? 0 : 1;
    ensure_shadow(c, A, prec, la);
    ensure_shadow(c, B, prec, lb);
    pa = reinterpret_cast<BlkIn>(A.lp[la].ptr.get());
    pb = reinterpret_cast<BlkIn>(B.lp[lb].ptr.get());
  }
  LIF_REQUIRE(!D || !D->holes, LIF_ERR_INVALID, "spgemm: the added term has holes");
  const int nb = A.nb;
  Bsr C = like(A);
  CsrView av, bv;
  if (ta) {
    av = transpose_view(c, A);
  } else {
    av.rp = A.row_ptr.get();
    av.col = A.col.get();
  }
  if (tb) {
    bv = transpose_view(c, B);
  } else {
    bv.rp = B.row_ptr.get();
    bv.col = B.col.get();
  }
  if (D) LIF_REQUIRE(D->nb == nb && D->b == A.b, LIF_ERR_INVALID, "spgemm: added term's shape differs");
  const int* drp = D ? D->row_ptr.get() : nullptr;
  const int* dcol = D ? D->col.get() : nullptr;
  C.row_ptr = DBuf<int>(c.pool, nb + 1);
  int64_t nnzc = 0, P = 0;  // capacities of the output and pair arrays
  bool planned = c.spec.on && c.spec.next < c.spec.caps.size() && c.spec.next < (size_t)Ctx::Spec::kSlots;
  int64_t exact_slot = -1;  // a slot of the planned sequence that this large product sizes exactly
  if (planned && c.spec.exact_large) {
    const auto& cp = c.spec.caps[c.spec.next];
    const double bytes = (double)std::min<int64_t>(cp[0], (int64_t)nb * nb) * A.b * A.b * sizeof(double) +
                         (double)cp[1] * sizeof(BlockPair);
    if (bytes > Ctx::Spec::kMaxBytes) {
      planned = false;
      exact_slot = (int64_t)c.spec.next++;
      c.spec.prec.push_back(prec);
    }
  }
  DBuf<int64_t> seg, prp;
  DBuf<BlockPair> pairs;
  DBuf<const double*> dsrc;
  auto alloc_outputs = [&]() {
    C.cap = nnzc;
    C.col = DBuf<int>(c.pool, (size_t)nnzc);
    seg = DBuf<int64_t>(c.pool, (size_t)nnzc + 1);
    pairs = DBuf<BlockPair>(c.pool, (size_t)P);
    dsrc = DBuf<const double*>(c.pool, D ? (size_t)nnzc : 0);
  };
  if (planned && symbolic_onepass_fits(nb)) {
    // sizes known in advance: count, scan and fill in one launch
    const size_t slot = c.spec.next++;
    nnzc = std::min<int64_t>(c.spec.caps[slot][0], (int64_t)nb * nb);
    P = c.spec.caps[slot][1];
    c.spec.prec.push_back(prec);
    C.nnzb = -1;
    alloc_outputs();
    launch_symbolic_onepass(c, av.rp, av.col, av.idx, bv.rp, bv.col, bv.idx, pa, pb, A.holes, B.holes,
                            drp, dcol, D ? D->ptrs() : nullptr, nb, nnzc, P, C.row_ptr.get(), C.col.get(),
                            seg.get(), pairs.get(), D ? dsrc.get() : nullptr, c.spec.sizes.get() + 2 * slot,
                            c.spec.overflow.get(), upper);
    return numeric_phase(c, std::move(C), ta, tb, tau, prec, alpha, D ? dsrc.get() : nullptr, gamma, keep_holes,
                         seg.get(), pairs.get(), nnzc, c.spec.overflow.get(), out_lp);
  }
  DBuf<int> cnt_c(c.pool, nb);
  DBuf<int64_t> cnt_p(c.pool, nb);
  launch_symbolic_count(c, av.rp, av.col, av.idx, bv.rp, bv.col, bv.idx, A.holes ? pa : nullptr,
                        B.holes ? pb : nullptr, drp, dcol, nb, cnt_c.get(), cnt_p.get(), upper);
  prp = DBuf<int64_t>(c.pool, nb + 1);
  if (planned) {
    const size_t slot = c.spec.next++;
    nnzc = std::min<int64_t>(c.spec.caps[slot][0], (int64_t)nb * nb);
    P = c.spec.caps[slot][1];
    scan_exclusive_pair_capped(c, cnt_c.get(), C.row_ptr.get(), cnt_p.get(), prp.get(), nb, nnzc, P,
                               c.spec.sizes.get() + 2 * slot, c.spec.overflow.get());
    c.spec.prec.push_back(prec);
    C.nnzb = -1;
  } else {
    scan_exclusive_pair(c, cnt_c.get(), C.row_ptr.get(), cnt_p.get(), prp.get(), nb);
    // the one read-back of a product: output and product counts, plus the
    // operands' block counts while only the device knows them
    int nnzc32 = 0, na = 0, nbk = 0;
    std::vector<Ctx::Read> reads{{&nnzc32, C.row_ptr.get() + nb, sizeof(int)},
                                 {&P, prp.get() + nb, sizeof(int64_t)}};
    const bool need_a = A.nnzb < 0, need_b = B.nnzb < 0 && &A != &B;
    if (need_a) reads.push_back({&na, A.live(), sizeof(int)});
    if (need_b) reads.push_back({&nbk, B.live(), sizeof(int)});
    c.d2h_batch(reads);
    if (need_a) A.nnzb = na;
    if (need_b) B.nnzb = nbk;
    nnzc = nnzc32;
    C.nnzb = nnzc;
    if (c.spec.record) c.spec.seen.push_back({nnzc, P});
    if (exact_slot >= 0) {
      if (c.spec.exact.size() <= (size_t)exact_slot) c.spec.exact.resize(exact_slot + 1, {-1, -1});
      c.spec.exact[exact_slot] = {nnzc, P};
    }
    if (exact_slot < 0) {  // a slot's statistics are counted once its sequence is kept
      c.stats.products += P;
      count_symbolic(c, nnzc, P, nb);
      const double fl = 2.0 * (double)C.b * C.b * C.b * (double)P;
      c.stats.flops += fl;
      if (prec != LIF_FP64) c.stats.flops_lowp += fl;
      if (prec == LIF_MIXED_FP32) c.stats.flops_f32 += fl;
    }
  }
  const double dev = (double)c.device_bytes(), pair_bytes = (double)P * sizeof(BlockPair);
  if (verbose() && (double)nnzc * A.b * A.b * sizeof(double) + pair_bytes > double(1u << 30))
    std::fprintf(stderr, "[lif]   product%s%s: %lld output blocks, %lld block products, in use %.2f GiB\n",
                 ta ? " A^T" : " A", tb ? " B^T" : " B", (long long)nnzc, (long long)P,
                 c.pool->in_use() / 1073741824.0);
  if (!planned && keep_holes && tau > 0.0 && nnzc > 0 && compact_output(c, nnzc, A.b) &&
      pair_bytes > std::min(kPairPanelBytes, dev / 512.0) &&
      (pair_bytes > dev / 64.0 || (double)c.pool->reserved() + pair_bytes > 0.5 * dev)) {
    // A large pair list: built and consumed one panel of block rows at a
    // time (a pair list of at most the panel budget, except a single row
    // above it), each panel's output compacted as it is computed.
    const int64_t budget = std::max<int64_t>(1, (int64_t)(std::min(kPairPanelBytes, dev / 512.0) / sizeof(BlockPair)));
    P = 0;  // no whole pair list
    alloc_outputs();
    C.blk = DBuf<const double*>(c.pool, (size_t)nnzc);
    C.holes = true;
    std::vector<int> hrp(nb + 1);
    std::vector<int64_t> hpp(nb + 1);
    c.d2h(hrp.data(), C.row_ptr.get(), sizeof(int) * (nb + 1));
    c.d2h(hpp.data(), prp.get(), sizeof(int64_t) * (nb + 1));
    Epilogue epi;
    epi.alpha = alpha;
    epi.gamma = gamma;
    epi.dsrc = D ? dsrc.get() : nullptr;
    epi.rows = C.row_ptr.get();
    epi.nrows = nb;
    epi.drop = true;
    epi.tau = tau;
    for (int r0 = 0; r0 < nb;) {
      int r1 = r0 + 1;
      while (r1 < nb && hpp[r1 + 1] - hpp[r0] <= budget) ++r1;
      const int64_t base = hpp[r0], np = hpp[r1] - base;
      if (hrp[r1] > hrp[r0]) {
        DBuf<BlockPair> pp(c.pool, (size_t)std::max<int64_t>(np, 1));
        // segment values stay global pair indices: the panel's pairs are
        // addressed through a pointer shifted back by the panel's first one
        BlockPair* shifted = reinterpret_cast<BlockPair*>(reinterpret_cast<uintptr_t>(pp.get()) -
                                                          (uintptr_t)base * sizeof(BlockPair));
        launch_symbolic_fill(c, av.rp, av.col, av.idx, bv.rp, bv.col, bv.idx, pa, pb, A.holes, B.holes, drp, dcol,
                             D ? D->ptrs() : nullptr, nb, C.row_ptr.get(), prp.get(), C.col.get(), seg.get(), shifted,
                             D ? dsrc.get() : nullptr, upper, r0, r1 - r0);
        numeric_compacted(c, C, prec, ta, tb, seg.get(), shifted, hrp[r0], hrp[r1], epi);
        ++c.stats.panels;
      }
      r0 = r1;
    }
    return C;
  }
  alloc_outputs();
  if (nnzc)
    launch_symbolic_fill(c, av.rp, av.col, av.idx, bv.rp, bv.col, bv.idx, pa, pb, A.holes, B.holes,
                         drp, dcol, D ? D->ptrs() : nullptr, nb, C.row_ptr.get(), prp.get(), C.col.get(), seg.get(),
                         pairs.get(), D ? dsrc.get() : nullptr, upper);
  return numeric_phase(c, std::move(C), ta, tb, tau, prec, alpha, D ? dsrc.get() : nullptr, gamma, keep_holes,
                       seg.get(), pairs.get(), nnzc, nullptr, out_lp);
}

}  // namespace

Bsr spgemm(Ctx& c, const Bsr& A, bool ta, const Bsr& B, bool tb, double tau, int prec, double alpha,
           const Bsr* D, double gamma, bool keep_holes, bool out_lp, bool upper) {
  Bsr C = spgemm_body(c, A, ta, B, tb, tau, prec, alpha, D, gamma, keep_holes, out_lp, upper);
  // with an operand known to be empty only the scaled added term remains
  const bool scaling = A.nnzb == 0 || B.nnzb == 0;
  task_after(c, C, !scaling, {&A, &B, D});
  return C;
}

namespace {

Bsr union_sum(Ctx& c, const Bsr* const src[3], const double coef[3], double gamma, const unsigned char* diag_on) {
  const Bsr* ref = nullptr;
  for (int t = 0; t < 3; ++t)
    if (src[t] && !ref) ref = src[t];
  Bsr C;
  C.n = ref ? ref->n : c.n;
  C.b = ref ? ref->b : c.b;
  C.nb = ref ? ref->nb : c.nb;
  const int nb = C.nb;
  const int* rp[3];
  const int* col[3];
  BlkIn val[3], hole[3];
  int64_t cap = diag_on ? nb : 0;
  // blocks that need new values: those of scaled operands, those present in
  // two or more unscaled operands (at most their total minus the largest),
  // and the identity's diagonal blocks; the rest are shared
  int64_t computed = diag_on ? nb : 0, unit_sum = 0, unit_max = 0;
  for (int t = 0; t < 3; ++t) {
    rp[t] = src[t] ? src[t]->row_ptr.get() : nullptr;
    col[t] = src[t] ? src[t]->col.get() : nullptr;
    val[t] = src[t] ? src[t]->ptrs() : nullptr;
    hole[t] = src[t] && src[t]->holes ? src[t]->ptrs() : nullptr;
    if (!src[t]) continue;
    cap += src[t]->bound();
    if (coef[t] == 1.0) {
      unit_sum += src[t]->bound();
      unit_max = std::max(unit_max, src[t]->bound());
    } else {
      computed += src[t]->bound();
    }
    C.share_store(*src[t]);
  }
  cap = std::min<int64_t>(cap, (int64_t)nb * nb);
  computed = std::min<int64_t>(computed + unit_sum - unit_max, cap);
  if (verbose() && (double)computed * C.b * C.b * sizeof(double) > double(1u << 30))
    std::fprintf(stderr, "[lif]   sum: %lld blocks at most, %lld computed at most, in use %.2f GiB\n", (long long)cap,
                 (long long)computed, c.pool->in_use() / 1073741824.0);
  C.nnzb = -1;
  C.cap = cap;
  C.row_ptr = DBuf<int>(c.pool, nb + 1);
  DBuf<int> slot(c.pool, 1);
  C.col = DBuf<int>(c.pool, (size_t)cap);
  DBuf<int> ix(c.pool, (size_t)cap * 3), rowof(c.pool, (size_t)cap);
  DBuf<unsigned char> id(c.pool, (size_t)cap);
  C.blk = DBuf<const double*>(c.pool, (size_t)cap);
  if (union_onepass_fits(nb)) {
    // pattern and the blocks taken unchanged in one launch, then values only
    // for the blocks that need them.  The bound on those can be far above
    // their number (operands with holes count their dropped blocks, and
    // operands with disjoint patterns share every block): above a gigabyte
    // the store waits for the count, one read-back.
    const bool exact = exact_store_pays(c, computed, C.b);
    Store st;
    if (!exact) {
      st = new_store(c, computed, C.b);
      C.store.push_back(st);
    }
    DBuf<int> list(c.pool, (size_t)std::max<int64_t>(computed, 1)), ncomp(c.pool, 1);
    launch_union3_onepass(c, rp, col, hole, val, coef, diag_on, C.row_ptr.get(), nb, C.col.get(), ix.get(), cap,
                          id.get(), rowof.get(), C.blk.get(), list.get(), ncomp.get());
    if (exact) {
      int nc = 0;
      c.d2h_batch({{&nc, ncomp.get(), sizeof(int)}});
      computed = nc;
      if (computed) {
        st = new_store(c, computed, C.b);
        C.store.push_back(st);
      }
    }
    if (computed)
      launch_axpby3_values(c, val, coef, ix.get(), cap, gamma, id.get(), rowof.get(), computed, C.b, C.n, st->get(),
                           nullptr, C.blk.get(), ncomp.get(), list.get());
    return C;
  }
  Store st = new_store(c, computed, C.b);
  C.store.push_back(st);
  {
    {
      DBuf<int> cnt(c.pool, nb);
      launch_union3(c, rp, col, hole, diag_on, nb, cnt.get(), slot.get());
      scan_exclusive_i32(c, cnt.get(), C.row_ptr.get(), nb);
    }
    if (cap)
      launch_union3_fill(c, rp, col, hole, diag_on, C.row_ptr.get(), nb, C.col.get(), ix.get(), cap, id.get(),
                         rowof.get());
  }
  if (cap)
    launch_axpby3_values(c, val, coef, ix.get(), cap, gamma, id.get(), rowof.get(), cap, C.b, C.n, st->get(),
                         slot.get(), C.blk.get(), C.live(), nullptr);
  return C;
}

}  // namespace

Bsr axpby(Ctx& c, double alpha, const Bsr* A, double beta, const Bsr* B, double gamma,
          const unsigned char* diag_on) {
  const Bsr* src[3] = {A, B, nullptr};
  const double coef[3] = {alpha, beta, 0.0};
  Bsr R = union_sum(c, src, coef, gamma, diag_on);
  task_after(c, R, false, {A, B});
  return R;
}

Bsr axpby3(Ctx& c, double alpha, const Bsr* A, double beta, const Bsr* B, double kappa, const Bsr* C) {
  const Bsr* src[3] = {A, B, C};
  const double coef[3] = {alpha, beta, kappa};
  Bsr R = union_sum(c, src, coef, 0.0, nullptr);
  task_after(c, R, false, {A, B, C});
  return R;
}

Bsr filter(Ctx& c, const Bsr& A, const int* rlab, const int* clab, int mode) {
  const int nb = A.nb;
  Bsr C = like(A);
  C.nnzb = -1;
  C.cap = A.bound();
  C.holes = A.holes;  // dropped blocks pass as null pointers, for products and sums
  C.row_ptr = DBuf<int>(c.pool, nb + 1);
  launch_filter_count_scan(c, A.row_ptr.get(), A.col.get(), rlab, clab ? clab : rlab, mode, nb, C.row_ptr.get());
  C.col = DBuf<int>(c.pool, (size_t)C.cap);
  DBuf<int> src(c.pool, (size_t)C.cap);
  C.blk = DBuf<const double*>(c.pool, (size_t)C.cap);
  C.share_store(A);
  if (C.cap) {
    launch_filter_fill(c, A.row_ptr.get(), A.col.get(), rlab, clab ? clab : rlab, mode, C.row_ptr.get(), nb,
                       C.col.get(), src.get());
    launch_gather_ptrs(c, A.ptrs(), src.get(), C.cap, C.blk.get(), C.live());
  }
  return C;
}

Bsr intersect(Ctx& c, const Bsr& A, const Bsr& R) {
  no_holes(A, "intersect");
  const int nb = A.nb;
  Bsr C = like(A);
  C.nnzb = -1;
  C.cap = A.bound();
  C.row_ptr = DBuf<int>(c.pool, nb + 1);
  launch_intersect_count_scan(c, A.row_ptr.get(), A.col.get(), R.row_ptr.get(), R.col.get(), nb, C.row_ptr.get());
  C.col = DBuf<int>(c.pool, (size_t)C.cap);
  DBuf<int> src(c.pool, (size_t)C.cap);
  C.blk = DBuf<const double*>(c.pool, (size_t)C.cap);
  C.share_store(A);
  if (C.cap) {
    launch_intersect(c, A.row_ptr.get(), A.col.get(), R.row_ptr.get(), R.col.get(), nb, nullptr, C.row_ptr.get(),
                     C.col.get(), src.get());
    launch_gather_ptrs(c, A.ptrs(), src.get(), C.cap, C.blk.get(), C.live());
  }
  return C;
}

Bsr phi_upper(Ctx& c, const Bsr& W) {
  no_holes(W, "phi_upper");
  std::vector<int> idx(W.nb);
  for (int i = 0; i < W.nb; ++i) idx[i] = i;
  DBuf<int> d_idx(c.pool, W.nb);
  h2d(c, d_idx.get(), idx.data(), W.nb);
  Bsr U = filter(c, W, d_idx.get(), d_idx.get(), 3);
  DBuf<int> rowof(c.pool, (size_t)std::max<int64_t>(U.cap, 1));
  launch_block_row_of(c, U.row_ptr.get(), U.nb, U.cap, rowof.get());
  Store st = new_store(c, U.nb, U.b);  // the new diagonal blocks, slot = block row
  U.store.push_back(st);
  launch_phi_diag(c, rowof.get(), U.col.get(), U.cap, U.b, st->get(), U.blk.get(), U.live());
  c.sync();  // idx goes out of scope
  return U;
}

double gershgorin(Ctx& c, const Bsr& A) {
  no_holes(A, "gershgorin");
  DBuf<double> rowmax(c.pool, A.nb), mx(c.pool, 1);
  launch_gershgorin(c, A.row_ptr.get(), A.ptrs(), A.nb, A.b, rowmax.get());
  launch_max_reduce(c, rowmax.get(), A.nb, mx.get());
  return read1(c, mx.get());
}

std::vector<double> node_sumsq(Ctx& c, const Bsr& A, const int* rlo, const int* rhi, int nseg,
                               const std::vector<Ctx::Read>& extra) {
  no_holes(A, "node_sumsq");
  std::vector<double> out(nseg, 0.0);
  if (nseg == 0) {
    if (!extra.empty()) c.d2h_batch(extra);
    return out;
  }
  DBuf<double> ss(c.pool, (size_t)std::max<int64_t>(A.bound(), 1)), seg(c.pool, nseg);
  launch_block_sumsq(c, A.ptrs(), A.bound(), A.b, ss.get(), false, A.live());
  launch_segment_sum(c, ss.get(), A.row_ptr.get(), rlo, rhi, nseg, seg.get());
  int na = 0;
  std::vector<Ctx::Read> reads;
  for (int s = 0; s < nseg; s += 8)
    reads.push_back({out.data() + s, seg.get() + s, sizeof(double) * (size_t)std::min(8, nseg - s)});
  const bool need = A.nnzb < 0;
  if (need) reads.push_back({&na, A.live(), sizeof(int)});
  int lb_fail = 0;
  if (c.lb_fail.get()) reads.push_back({&lb_fail, c.lb_fail.get(), sizeof(int)});
  reads.insert(reads.end(), extra.begin(), extra.end());
  c.d2h_batch(reads);
  LIF_REQUIRE(!lb_fail, LIF_ERR_HIP, "a single-pass scan gave up waiting for a lower row (workgroups started out "
                                     "of order); results of this call are invalid");
  if (need) A.nnzb = na;
  return out;
}

}  // namespace lif
