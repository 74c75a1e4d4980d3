// Block-sparse operations on device block-CSR matrices.  Each operation
// allocates its outputs from the handle's pool, queues its kernels on the
// handle's stream and reads back only the sizes it needs to allocate.
#include <algorithm>

#include "common.h"

namespace lif {

size_t symbolic_lds_bytes(int nb, bool fill);

namespace {

template <typename T>
T read1(Ctx& c, const T* dev) {
  T v;
  c.d2h(&v, dev, sizeof(T));
  return v;
}

}  // namespace

Bsr bsr_empty(Ctx& c, int64_t n, int b) {
  Bsr A;
  A.n = n;
  A.b = b;
  A.nb = (int)((n + b - 1) / b);
  A.nnzb = 0;
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
  const hipMemcpyKind kind = in.on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  DBuf<int> brow(c.pool, (size_t)in.nnzb);
  A.col = DBuf<int>(c.pool, (size_t)in.nnzb);
  A.val = DBuf<double>(c.pool, (size_t)in.nnzb * in.b * in.b);
  if (in.nnzb) {
    LIF_HIP(hipMemcpyAsync(brow.get(), in.brow, in.nnzb * sizeof(int), kind, c.stream));
    LIF_HIP(hipMemcpyAsync(A.col.get(), in.bcol, in.nnzb * sizeof(int), kind, c.stream));
    LIF_HIP(hipMemcpyAsync(A.val.get(), in.vals, in.nnzb * (size_t)in.b * in.b * sizeof(double), kind, c.stream));
  }
  A.row_ptr = DBuf<int>(c.pool, A.nb + 1);
  launch_row_ptr_from_rows(c, brow.get(), in.nnzb, A.nb, A.row_ptr.get());
  return A;
}

void bsr_to_blocks(Ctx& c, const Bsr& A, int32_t* brow, int32_t* bcol, double* vals, bool on_device) {
  if (A.nnzb == 0) return;
  DBuf<int> rows(c.pool, (size_t)A.nnzb);
  launch_block_row_of(c, A.row_ptr.get(), A.nb, A.nnzb, rows.get());
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  LIF_HIP(hipMemcpyAsync(brow, rows.get(), A.nnzb * sizeof(int), kind, c.stream));
  LIF_HIP(hipMemcpyAsync(bcol, A.col.get(), A.nnzb * sizeof(int), kind, c.stream));
  LIF_HIP(hipMemcpyAsync(vals, A.val.get(), A.nnzb * (size_t)A.b * A.b * sizeof(double), kind, c.stream));
  c.sync();
}

Bsr copy(Ctx& c, const Bsr& A) {
  Bsr B;
  B.n = A.n;
  B.b = A.b;
  B.nb = A.nb;
  B.nnzb = A.nnzb;
  B.row_ptr = DBuf<int>(c.pool, A.nb + 1);
  B.col = DBuf<int>(c.pool, (size_t)A.nnzb);
  B.val = DBuf<double>(c.pool, (size_t)A.nnzb * A.b * A.b);
  LIF_HIP(hipMemcpyAsync(B.row_ptr.get(), A.row_ptr.get(), (A.nb + 1) * sizeof(int), hipMemcpyDeviceToDevice,
                         c.stream));
  if (A.nnzb) {
    LIF_HIP(hipMemcpyAsync(B.col.get(), A.col.get(), A.nnzb * sizeof(int), hipMemcpyDeviceToDevice, c.stream));
    LIF_HIP(hipMemcpyAsync(B.val.get(), A.val.get(), A.nnzb * (size_t)A.b * A.b * sizeof(double),
                           hipMemcpyDeviceToDevice, c.stream));
  }
  return B;
}

DBuf<double> block_norms(Ctx& c, const Bsr& A) {
  DBuf<double> nrm(c.pool, (size_t)A.nnzb);
  launch_block_sumsq(c, A.val.get(), A.nnzb, A.b, nrm.get(), true);
  return nrm;
}

// Sec. 5 truncation: drop blocks with Frobenius norm < tau, keep the order.
Bsr truncate(Ctx& c, Bsr&& A, const double* norms, double tau) {
  if (tau <= 0.0 || A.nnzb == 0) return std::move(A);
  DBuf<int> cnt(c.pool, A.nb);
  launch_keep_counts(c, A.row_ptr.get(), norms, tau, A.nb, cnt.get());
  DBuf<int> nrp(c.pool, A.nb + 1);
  scan_exclusive_i32(c, cnt.get(), nrp.get(), A.nb);
  const int nnz = read1(c, nrp.get() + A.nb);
  if (nnz == A.nnzb) return std::move(A);
  Bsr B;
  B.n = A.n;
  B.b = A.b;
  B.nb = A.nb;
  B.nnzb = nnz;
  B.row_ptr = std::move(nrp);
  B.col = DBuf<int>(c.pool, (size_t)nnz);
  DBuf<int> src(c.pool, (size_t)nnz);
  launch_compact_index(c, A.row_ptr.get(), A.col.get(), norms, tau, B.row_ptr.get(), A.nb, B.col.get(), src.get());
  B.val = DBuf<double>(c.pool, (size_t)nnz * A.b * A.b);
  launch_gather_blocks(c, A.val.get(), src.get(), nnz, A.b, B.val.get());
  return B;
}

CsrView transpose_view(Ctx& c, const Bsr& A) {
  CsrView v;
  const int nb = A.nb;
  DBuf<int> cnt(c.pool, nb);
  launch_fill_i32(c, cnt.get(), 0, nb);
  launch_transpose_counts(c, A.col.get(), A.nnzb, cnt.get());
  v.own_rp = DBuf<int>(c.pool, nb + 1);
  scan_exclusive_i32(c, cnt.get(), v.own_rp.get(), nb);
  launch_fill_i32(c, cnt.get(), 0, nb);
  DBuf<int> tcol(c.pool, (size_t)A.nnzb), tsrc(c.pool, (size_t)A.nnzb);
  if (A.nnzb) {
    launch_transpose_fill(c, A.row_ptr.get(), A.col.get(), v.own_rp.get(), nb, cnt.get(), tcol.get(), tsrc.get());
  }
  v.own_col = DBuf<int>(c.pool, (size_t)A.nnzb);
  v.own_idx = DBuf<int>(c.pool, (size_t)A.nnzb);
  if (A.nnzb) {
    launch_transpose_sort(c, v.own_rp.get(), nb, tcol.get(), tsrc.get(), v.own_col.get(), v.own_idx.get());
  }
  v.rp = v.own_rp.get();
  v.col = v.own_col.get();
  v.idx = v.own_idx.get();
  return v;
}

Bsr transpose(Ctx& c, const Bsr& A) {
  CsrView v = transpose_view(c, A);
  Bsr T;
  T.n = A.n;
  T.b = A.b;
  T.nb = A.nb;
  T.nnzb = A.nnzb;
  T.row_ptr = std::move(v.own_rp);
  T.col = std::move(v.own_col);
  T.val = DBuf<double>(c.pool, (size_t)A.nnzb * A.b * A.b);
  launch_transpose_blocks(c, A.val.get(), v.own_idx.get(), A.nnzb, A.b, T.val.get());
  return T;
}

Bsr spgemm(Ctx& c, const Bsr& A, bool ta, const Bsr& B, bool tb, double tau, int prec) {
  LIF_REQUIRE(A.nb == B.nb && A.b == B.b, LIF_ERR_INVALID, "spgemm: operand shapes differ");
  const int nb = A.nb;
  Bsr C;
  C.n = A.n;
  C.b = A.b;
  C.nb = nb;
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
  DBuf<int> cnt_c(c.pool, nb);
  DBuf<int64_t> cnt_p(c.pool, nb);
  launch_symbolic_count(c, av.rp, av.col, bv.rp, bv.col, nb, cnt_c.get(), cnt_p.get());
  C.row_ptr = DBuf<int>(c.pool, nb + 1);
  DBuf<int64_t> prp(c.pool, nb + 1);
  scan_exclusive_i32(c, cnt_c.get(), C.row_ptr.get(), nb);
  scan_exclusive_i64(c, cnt_p.get(), prp.get(), nb);
  int nnzc32 = 0;
  int64_t P = 0;
  c.d2h2(&nnzc32, C.row_ptr.get() + nb, sizeof(int), &P, prp.get() + nb, sizeof(int64_t));
  const int64_t nnzc = nnzc32;
  C.nnzb = nnzc;
  C.col = DBuf<int>(c.pool, (size_t)nnzc);
  DBuf<int64_t> seg(c.pool, (size_t)nnzc + 1);
  DBuf<int2> pairs(c.pool, (size_t)P);
  if (nnzc) {
    launch_symbolic_fill(c, av.rp, av.col, av.idx, bv.rp, bv.col, bv.idx, nb, C.row_ptr.get(), prp.get(),
                         C.col.get(), seg.get(), pairs.get());
    LIF_HIP(hipMemcpyAsync(seg.get() + nnzc, prp.get() + nb, sizeof(int64_t), hipMemcpyDeviceToDevice, c.stream));
  }
  C.val = DBuf<double>(c.pool, (size_t)nnzc * C.b * C.b);
  DBuf<double> nrm(c.pool, (size_t)nnzc);
  launch_numeric(c, prec, A.val.get(), B.val.get(), ta, tb, seg.get(), pairs.get(), nnzc, C.b, C.val.get(),
                 nrm.get());
  c.stats.products += P;
  const double fl = 2.0 * (double)C.b * C.b * C.b * (double)P;
  c.stats.flops += fl;
  if (prec != LIF_FP64) c.stats.flops_lowp += fl;
  return truncate(c, std::move(C), nrm.get(), tau);
}

Bsr axpby(Ctx& c, double alpha, const Bsr* A, double beta, const Bsr* B, double gamma,
          const unsigned char* diag_on) {
  const Bsr* ref = A ? A : B;
  const int nb = ref ? ref->nb : c.nb;
  Bsr C;
  C.n = ref ? ref->n : c.n;
  C.b = ref ? ref->b : c.b;
  C.nb = nb;
  const int* ra = A ? A->row_ptr.get() : nullptr;
  const int* ca = A ? A->col.get() : nullptr;
  const int* rb = B ? B->row_ptr.get() : nullptr;
  const int* cb = B ? B->col.get() : nullptr;
  DBuf<int> cnt(c.pool, nb);
  launch_union_counts(c, ra, ca, rb, cb, diag_on, nb, cnt.get());
  C.row_ptr = DBuf<int>(c.pool, nb + 1);
  scan_exclusive_i32(c, cnt.get(), C.row_ptr.get(), nb);
  const int nnz = read1(c, C.row_ptr.get() + nb);
  C.nnzb = nnz;
  C.col = DBuf<int>(c.pool, (size_t)nnz);
  DBuf<int> ia(c.pool, (size_t)nnz), ib(c.pool, (size_t)nnz), rowof(c.pool, (size_t)nnz);
  DBuf<unsigned char> id(c.pool, (size_t)nnz);
  C.val = DBuf<double>(c.pool, (size_t)nnz * C.b * C.b);
  if (nnz) {
    launch_union_fill(c, ra, ca, rb, cb, diag_on, C.row_ptr.get(), nb, C.col.get(), ia.get(), ib.get(), id.get());
    launch_block_row_of(c, C.row_ptr.get(), nb, nnz, rowof.get());
    launch_axpby_values(c, alpha, A ? A->val.get() : nullptr, ia.get(), beta, B ? B->val.get() : nullptr, ib.get(),
                        gamma, id.get(), rowof.get(), nnz, C.b, C.n, C.val.get());
  }
  return C;
}

Bsr filter(Ctx& c, const Bsr& A, const int* rlab, const int* clab, int mode) {
  const int nb = A.nb;
  Bsr C;
  C.n = A.n;
  C.b = A.b;
  C.nb = nb;
  DBuf<int> cnt(c.pool, nb);
  launch_filter_counts(c, A.row_ptr.get(), A.col.get(), rlab, clab ? clab : rlab, mode, nb, cnt.get());
  C.row_ptr = DBuf<int>(c.pool, nb + 1);
  scan_exclusive_i32(c, cnt.get(), C.row_ptr.get(), nb);
  const int nnz = read1(c, C.row_ptr.get() + nb);
  C.nnzb = nnz;
  C.col = DBuf<int>(c.pool, (size_t)nnz);
  DBuf<int> src(c.pool, (size_t)nnz);
  C.val = DBuf<double>(c.pool, (size_t)nnz * C.b * C.b);
  if (nnz) {
    launch_filter_fill(c, A.row_ptr.get(), A.col.get(), rlab, clab ? clab : rlab, mode, C.row_ptr.get(), nb,
                       C.col.get(), src.get());
    launch_gather_blocks(c, A.val.get(), src.get(), nnz, C.b, C.val.get());
  }
  return C;
}

double gershgorin(Ctx& c, const Bsr& A) {
  DBuf<double> rowmax(c.pool, A.nb), mx(c.pool, 1);
  launch_gershgorin(c, A.row_ptr.get(), A.val.get(), A.nb, A.b, rowmax.get());
  launch_max_reduce(c, rowmax.get(), A.nb, mx.get());
  return read1(c, mx.get());
}

std::vector<double> node_sumsq(Ctx& c, const Bsr& A, const int* rlo, const int* rhi, int nseg) {
  std::vector<double> out(nseg, 0.0);
  if (nseg == 0) return out;
  DBuf<double> ss(c.pool, (size_t)std::max<int64_t>(A.nnzb, 1)), seg(c.pool, nseg);
  launch_block_sumsq(c, A.val.get(), A.nnzb, A.b, ss.get(), false);
  launch_segment_sum(c, ss.get(), A.row_ptr.get(), rlo, rhi, nseg, seg.get());
  c.d2h(out.data(), seg.get(), nseg * sizeof(double));
  return out;
}

}  // namespace lif
