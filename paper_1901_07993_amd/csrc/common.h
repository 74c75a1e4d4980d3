// Internal declarations of the inverse-factorization library: device memory
// pool, RAII device buffers, the device block-CSR matrix and the launchers of
// every kernel.  Host code only; kernels live in the *.hip files.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdint>
#include <cstring>
#include <initializer_list>
#include <map>
#include <memory>
#include <set>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "../../include/lif.h"

namespace lif {

struct Error : std::runtime_error {
  int status;
  Error(int s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define LIF_HIP(x)                                                                         \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess)                                                                  \
      throw ::lif::Error(LIF_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_));     \
  } while (0)

#define LIF_REQUIRE(cond, status, msg)          \
  do {                                          \
    if (!(cond)) throw ::lif::Error((status), (msg)); \
  } while (0)

// ---------------------------------------------------------------------------
// Device memory pool: caches freed allocations by exact rounded size so the
// refinement loop does not call hipMalloc/hipFree once warm.  All memory of a
// handle goes through one pool, which enforces the handle's byte cap.
// ---------------------------------------------------------------------------
// Device memory: a few large segments from hipMalloc, carved into buffers
// best-fit and merged again when freed, so that the changing sizes of
// products from one iteration to the next cost no hipMalloc / hipFree
// (each of those can take milliseconds for a large buffer).
class Pool {
 public:
  explicit Pool(uint64_t cap) : cap_(cap) {}
  // A pool over one fixed device region it does not own: every buffer is
  // carved from [base, base + bytes), nothing is ever requested from or
  // returned to HIP, and a request that does not fit fails with
  // LIF_ERR_OUT_OF_MEMORY.
  Pool(void* base, size_t bytes);
  ~Pool() { release_all(); }
  void* alloc(size_t bytes);
  void free(void* p);
  // Gives back the tail of a buffer beyond its first `bytes` (which the
  // device must no longer touch); false when the buffer keeps its size
  // (freed buffers are being held back, or nothing to give).
  bool shrink(void* p, size_t bytes);
  void trim();            // return wholly unused segments to HIP
  // While deferring, freed buffers are held back from reuse until
  // release_deferred(): work on two streams may still read a buffer the host
  // has released, and reuse is only safe after both streams have synchronized.
  void set_defer(bool on) { defer_ = on; }
  bool deferring() const { return defer_; }
  void release_deferred();
  uint64_t cap() const { return cap_; }  // 0: no cap
  uint64_t in_use() const { return in_use_; }
  uint64_t reserved() const { return reserved_; }
  uint64_t peak() const { return peak_; }
  void reset_peak() { peak_ = in_use_; }
  int64_t segments_allocated() const { return seg_allocs_; }

 private:
  struct Piece {
    size_t size;
    bool free;
    char* seg;  // base of the segment it lies in
  };
  // Buffers of at least kLarge bytes and smaller ones live in separate
  // segments, so that small long-lived buffers never pin a large segment.
  static constexpr size_t kLarge = size_t(64) << 20;
  int size_class(size_t r) const { return (!fixed_ && r >= kLarge) ? 1 : 0; }
  bool fixed_ = false;  // one region given at construction, not owned
  static size_t round(size_t bytes);
  bool grow(size_t need, int cls);
  void take(std::map<char*, Piece>::iterator it, size_t r);
  void release_all();
  uint64_t cap_;
  uint64_t in_use_ = 0, reserved_ = 0, peak_ = 0;
  uint64_t reserved_cls_[2] = {0, 0};
  int64_t seg_allocs_ = 0;
  std::map<char*, std::pair<size_t, int>> segs_;  // segment base -> (size, class)
  std::map<char*, Piece> pieces_;                 // every piece of every segment, by address
  std::set<std::pair<size_t, char*>> free_[2];    // free pieces of each class by (size, address)
  bool defer_ = false;
  std::vector<void*> deferred_;
};

template <typename T>
class DBuf {
 public:
  DBuf() = default;
  DBuf(Pool* pool, size_t n) : pool_(pool), n_(n) {
    p_ = n ? static_cast<T*>(pool->alloc(n * sizeof(T))) : nullptr;
  }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : pool_(o.pool_), p_(o.p_), n_(o.n_) { o.p_ = nullptr; o.n_ = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      reset();
      pool_ = o.pool_; p_ = o.p_; n_ = o.n_;
      o.p_ = nullptr; o.n_ = 0;
    }
    return *this;
  }
  ~DBuf() { reset(); }
  void reset() {
    if (p_ && pool_) pool_->free(p_);
    p_ = nullptr;
    n_ = 0;
  }
  T* get() const { return p_; }
  size_t size() const { return n_; }
  // keeps the first n elements and returns the rest to the pool
  void shrink(size_t n) {
    if (n == 0) {
      reset();
    } else if (n < n_ && p_ && pool_ && pool_->shrink(p_, n * sizeof(T))) {
      n_ = n;
    }
  }

 private:
  Pool* pool_ = nullptr;
  T* p_ = nullptr;
  size_t n_ = 0;
};

// ---------------------------------------------------------------------------
// Device block-CSR matrix: nb block rows, row_ptr[nb+1], col[nnzb] sorted
// within each row, blk[nnzb] pointers to row-major FP64 b x b blocks.
// ---------------------------------------------------------------------------
//
// The block count may be known only on the device (row_ptr[nb]): operations
// that cannot grow a matrix beyond a host-known bound (truncation, filters,
// sums) allocate that bound as capacity and leave nnzb = -1, so they need no
// device-to-host read.  Kernels that run over blocks take the device count
// and skip the tail of the capacity.
// Block pointer arrays (device): block e of a matrix is the b*b row-major
// doubles at blk[e].  A value block is written once by the kernel that
// creates it and only read afterwards, so matrices share blocks freely:
// truncation, filters and copies move pointers, and a sum reuses the blocks
// it takes unscaled from one operand.
// Loads through a pointer that was itself read from memory compile to flat
// loads, which count on both the vector-memory and the LDS counters, so the
// compiler waits for all outstanding ones before the first use; through a
// pointer cast to the global address space they are global loads, waited
// for one by one as their data is needed.
template <typename T>
__device__ __attribute__((always_inline)) inline const __attribute__((address_space(1))) T* gptr(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}

typedef const double* const* BlkIn;
typedef const double** BlkOut;
typedef std::shared_ptr<DBuf<double>> Store;

// The two operand blocks of one block product of a sparse product.
struct BlockPair {
  const double* a;
  const double* b;
};

struct Bsr {
  int64_t n = 0;
  int b = 0;
  int nb = 0;
  mutable int64_t nnzb = 0;  // exact block count, or -1 while only the device knows it
  int64_t cap = 0;           // blocks allocated in col and blk (>= the count)
  DBuf<int> row_ptr;
  DBuf<int> col;
  DBuf<const double*> blk;   // [cap] value block pointers
  std::vector<Store> store;  // value arrays the pointers point into (kept alive)
  // A product whose dropped blocks (norm below the threshold) were not
  // compacted away: their pointers are null and they count as absent.  Only
  // products, sums and transposed views read such a matrix.
  bool holes = false;
  // Task-graph shadow (the critical-path model of Sec. 3, where products,
  // sums, scalings, separate transposes and factorizations are tasks): the
  // longest chain of dependent tasks that ends in this matrix, and the
  // products on that chain.  Inputs start at 0; operations that are not
  // tasks (filters, truncation, compaction) pass the counts on.
  int cpl = 0;
  int cpl_products = 0;
  // Copies of the blocks in a product input precision (FP32 or BF16), one
  // per layout: [0] blocks as stored, [1] each block transposed.  ptr[e]
  // is block e's copy (null where blk[e] is null).  Made on first use by a
  // reduced-precision product, or written by the product that created the
  // matrix; anything that moves blk drops them.
  struct Shadow {
    int prec = LIF_FP64;  // LIF_FP64: no copy
    DBuf<const void*> ptr;
    Store store;
  };
  mutable Shadow lp[2];
  int64_t bound() const { return nnzb >= 0 ? nnzb : cap; }
  const int* live() const { return row_ptr.get() + nb; }  // device-side count
  BlkIn ptrs() const { return blk.get(); }
  void share_store(const Bsr& o) {
    for (const Store& s : o.store)
      if (std::find(store.begin(), store.end(), s) == store.end()) store.push_back(s);
  }
  // blocks held by the value arrays this matrix points into
  int64_t store_blocks() const {
    size_t d = 0;
    for (const Store& s : store) d += s->size();
    return b ? (int64_t)(d / ((size_t)b * b)) : 0;
  }
};

// Per-call statistics.
struct Stats {
  double flops = 0;
  double flops_lowp = 0;  // part of flops done with FP32/BF16 inputs
  int64_t products = 0;
  int64_t gemm_launches = 0;
  double gemm_ms = 0;
  double gemm_ms_lowp = 0;        // part of gemm_ms spent in FP32/BF16-input launches
  int64_t gemm_launches_lowp = 0;
  double flops_f32 = 0, gemm_ms_f32 = 0;  // the FP32-input part of the three above
  int64_t gemm_launches_f32 = 0;
  // timing level 2: the leaf factorizations and the symbolic phases, with the
  // algorithmic work of each -- the band-limited factorization's and the
  // dense inverse's flops; the symbolic phase's bytes (each block product
  // reads one column index of B and writes a 16-byte pair, each output block
  // a column index and a segment start; the row pointers)
  double leaf_ms = 0, leaf_flops = 0;
  double sym_ms = 0, sym_bytes = 0;
  int64_t leaf_launches = 0, sym_launches = 0;
  int redone = 0;  // presized iterations redone with exact sizes
  int cpl = 0;           // longest chain of dependent tasks so far (Bsr::cpl)
  int cpl_products = 0;  // products on it
  int64_t compacted = 0;  // products written as kept blocks only
  int64_t panels = 0;     // row panels of products built one pair list at a time
};

// Execution context shared by all operations of a handle.
struct Ctx {
  hipStream_t stream = nullptr;
  Pool* pool = nullptr;
  Stats stats;
  bool timing = false;
  int b = 64;
  int64_t n = 0;
  int nb = 0;
  // No host allocation through HIP (pinned staging, mapped read-back
  // buffer): reads go to the caller's host memory with plain copies, and
  // look-back words are cleared by a fill kernel (allocation-free entry point).
  bool no_host_alloc = false;
  // pinned host staging for small device->host reads
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  void* readback = nullptr;  // mapped pinned area written by the read-back kernel
  // per-block-row flags, all set (identity on every row)
  DBuf<unsigned char> ones;
  // Products sized in advance.  While `on`, spgemm takes its output and pair
  // capacities from caps[next] instead of reading the counts back, writes
  // the true counts to sizes[2 next .. 2 next + 1] and raises *overflow when
  // a capacity was short (the product then reads as empty, and the caller
  // redoes the work with exact sizes).  While `record` (and not `on`), the
  // counts spgemm reads back are appended to `seen`.
  struct Spec {
    static constexpr int kSlots = 32;
    bool on = false, record = false;
    size_t next = 0;
    std::vector<std::array<int64_t, 2>> caps, seen;
    std::vector<int> prec;  // precision of each sized-in-advance product
    // While exact_large, a product whose capacity would take more than
    // kMaxBytes is sized exactly even in a planned sequence (a read-back
    // costs little next to it, a margin costs gigabytes): exact[slot] holds
    // its counts, {-1, -1} for the planned slots.
    static constexpr double kMaxBytes = double(1u << 30);
    bool exact_large = false;  // set while memory is tight
    std::vector<std::array<int64_t, 2>> exact;
    DBuf<int64_t> sizes;
    DBuf<int> overflow;
  } spec;
  // State of the single-pass scans (look-back over groups of rows), one per
  // stream: published words (two arrays of `rows` per-row words, then two of
  // groups(rows) per-group words) and the epoch that tells this launch's
  // words from those of earlier ones.
  struct Lookback {
    static int groups(int rows) { return (rows + 63) / 64; }
    DBuf<unsigned long long> words;
    int rows = 0;
    unsigned epoch = 0;
    unsigned next_epoch() {
      epoch = (epoch + 1) & 0x3fffu;
      if (epoch == 0) epoch = 1;
      return epoch;
    }
  };
  std::map<hipStream_t, Lookback> lookback;
  Lookback& lookback_for(int rows);  // the current stream's, for `rows` rows
  // the word arrays of the current stream's look-back and a fresh epoch,
  // for one launch over `rows` rows
  struct LbWords {
    unsigned long long* ra = nullptr;  // per-row words, first value
    unsigned long long* rb = nullptr;  // per-row words, second value
    unsigned long long* ga = nullptr;  // per-group sums, first value
    unsigned long long* gb = nullptr;  // per-group sums, second value
    unsigned epoch = 0;
    int* fail = nullptr;  // raised by a row whose wait gave up
  };
  LbWords lookback_words(int rows);
  // raised on the device when a single-pass scan gave up waiting (its
  // result is wrong); checked with the refinement's norms
  DBuf<int> lb_fail;
  // events around leaf-GEMM launches (timing mode), resolved at flush_timing()
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
  std::vector<char> ev_lowp;  // per pending pair: the input precision of the launch (LIF_FP64 = 0: FP64)
  // per pending pair: what it timed (Timed::Gemm, Leaf or Symbolic)
  std::vector<char> ev_cat;
  enum Timed { Gemm = 0, Leaf = 1, Symbolic = 2 };
  // 1: every leaf-GEMM launch is timed; 2: also the leaf factorizations and
  // the symbolic phases (more events per step; for per-kernel rooflines)
  int timing_level = 0;
  // an event recorded on the current stream when timing is at least `level`
  hipEvent_t timed_begin(int level);
  // closes the interval opened by timed_begin (a null begin: nothing)
  void timed_end(hipEvent_t e0, Timed what);
  std::vector<hipEvent_t> ev_free;

  hipEvent_t take_event();
  // a second stream (default priority) for work that may overlap the main
  // stream's, ordered against it with events; created on first use
  hipStream_t side = nullptr;
  std::vector<hipEvent_t> order_events;
  hipStream_t side_stream();
  // device memory the handle may use: the GPU's (queried once), or the
  // pool's cap when smaller.  Sizes the large-problem policies: when an
  // iteration's buffers go to one stream and are freed early, which
  // products are written compacted, and the panels of the residual.
  uint64_t device_bytes();
  uint64_t device_total = 0;
  hipEvent_t order_event(size_t i);  // the i-th reusable ordering event
  // `waiter` waits for the work queued so far on `signaler`
  void stream_after(hipStream_t waiter, hipStream_t signaler);
  std::vector<hipEvent_t> ring_events;
  size_t next_order = 0;
  void flush_timing();
  void sync() { LIF_HIP(hipStreamSynchronize(stream)); }
  // copy `bytes` from device `src` through the pinned buffer; synchronizes
  void d2h(void* dst, const void* src, size_t bytes);
  // several small reads (at most 64 bytes each) with one synchronization
  struct Read {
    void* dst;
    const void* src;
    size_t bytes;
  };
  void d2h_batch(const std::vector<Read>& reads);
  ~Ctx();
};

// LIF_VERBOSE set in the environment: one line per refinement iteration and
// per large product on stderr (sizes, memory), for following long runs.
bool verbose();

// The symbolic phase's algorithmic bytes of one product (Stats::sym_bytes).
inline void count_symbolic(Ctx& c, int64_t nnzc, int64_t pairs, int nb) {
  c.stats.sym_bytes += 20.0 * (double)pairs + 12.0 * (double)nnzc + 8.0 * (double)(nb + 1);
}

// Launches within the scope go to stream s.
struct StreamScope {
  Ctx& c;
  hipStream_t keep;
  StreamScope(Ctx& ctx, hipStream_t s) : c(ctx), keep(ctx.stream) { c.stream = s; }
  ~StreamScope() { c.stream = keep; }
  StreamScope(const StreamScope&) = delete;
  StreamScope& operator=(const StreamScope&) = delete;
};

// Buffers freed within the scope are reused only after release(), which the
// caller invokes once the host has synchronized with every stream; on an
// early exit the destructor synchronizes the device first.
struct DeferFrees {
  Ctx& c;
  bool active = true;
  explicit DeferFrees(Ctx& ctx) : c(ctx) { c.pool->set_defer(true); }
  void release() {
    if (!active) return;
    c.pool->set_defer(false);
    c.pool->release_deferred();
    active = false;
  }
  ~DeferFrees() {
    if (!active) return;
    (void)hipDeviceSynchronize();
    release();
  }
  DeferFrees(const DeferFrees&) = delete;
  DeferFrees& operator=(const DeferFrees&) = delete;
};

// ---------------------------------------------------------------------------
// Launchers (defined in the .hip files).  All enqueue on ctx.stream.
// ---------------------------------------------------------------------------

// scan.hip
// out[0] = 0, out[i+1] = out[i] + in[i] for i < count
void scan_exclusive_i32(Ctx& c, const int* in, int* out, int count);
// both scans of the symbolic phase in one launch
void scan_exclusive_pair(Ctx& c, const int* in32, int* out32, const int64_t* in64, int64_t* out64, int count);
// the same against capacities fixed in advance: the totals go to sizes[0..1];
// if either exceeds its capacity both outputs are zeroed (an empty product)
// and *overflow is set to 1
void scan_exclusive_pair_capped(Ctx& c, const int* in32, int* out32, const int64_t* in64, int64_t* out64, int count,
                                int64_t cap32, int64_t cap64, int64_t* sizes, int* overflow);

// bsr.hip
void launch_row_ptr_from_rows(Ctx& c, const int* brow, int64_t nnzb, int nb, int* row_ptr);
void launch_block_sumsq(Ctx& c, BlkIn blk, int64_t nnzb, int b, double* out, bool take_sqrt, const int* live);
// out[e] = blk[src[e]]
void launch_gather_ptrs(Ctx& c, BlkIn blk, const int* src, int64_t nnzb, BlkOut out, const int* live);
// out[e] = base + e b^2, e < count
void launch_fill_ptrs(Ctx& c, BlkOut out, const double* base, int b, int64_t count);
// the blocks' values, contiguous: block e to out + e b^2
void launch_gather_values(Ctx& c, BlkIn blk, int64_t nnzb, int b, double* out, const int* live);
void launch_gershgorin(Ctx& c, const int* row_ptr, BlkIn blk, int nb, int b, double* row_max);
void launch_max_reduce(Ctx& c, const double* in, int count, double* out);
// per-row counts of the union; also zeroes *slot (nullable) for the values pass
// hole[t]: the block pointers of an operand with holes (null otherwise);
// its null blocks are skipped
void launch_union3(Ctx& c, const int* const rp[3], const int* const col[3], const BlkIn hole[3],
                   const unsigned char* diag_on, int nb, int* counts, int* slot);
void launch_union3_fill(Ctx& c, const int* const rp[3], const int* const col[3], const BlkIn hole[3],
                        const unsigned char* diag_on, const int* rc, int nb, int* cc, int* ix, int64_t stride,
                        unsigned char* id, int* rowof);
// counts, row pointers (written to rc[0..nb]) and fill in one launch, with
// the row counts' prefix sums by look-back.  Output blocks taken unchanged
// from one operand (coefficient 1, no identity term) get that operand's
// pointer in out; the others are listed, in row order, in list[0..*ncomp)
// for the values pass.  Only for nb with union_onepass_fits(nb).
bool union_onepass_fits(int nb);
void launch_union3_onepass(Ctx& c, const int* const rp[3], const int* const col[3], const BlkIn hole[3],
                           const BlkIn val[3], const double coef[3], const unsigned char* diag_on, int* rc, int nb,
                           int* cc, int* ix, int64_t stride, unsigned char* id, int* rowof, BlkOut out, int* list,
                           int* ncomp);
void launch_keep_count_scan(Ctx& c, const int* row_ptr, const double* norms, double tau, int nb, int* out_rp);
void launch_filter_count_scan(Ctx& c, const int* row_ptr, const int* col, const int* rlab, const int* clab, int mode,
                              int nb, int* out_rp);
void launch_intersect_count_scan(Ctx& c, const int* ra, const int* ca, const int* rr, const int* cr, int nb,
                                 int* out_rp);
void launch_compact_gather(Ctx& c, const int* row_ptr, int nb, const int* col, const double* norms, double tau,
                           const int* new_row_ptr, BlkIn blk, int64_t nnzb, int* new_col, BlkOut new_blk);
// out block e = sum_t coef[t] v[t][ix[t][e]] (+ gamma I on the real rows of
// flagged diagonal blocks); computed blocks take slots of `store` from the
// counter *slot, blocks taken unscaled from one operand are shared.  With
// `list` (nullable): only the blocks e = list[w], w < *live, each computed
// into slot w (nnzb is then the list's capacity).
void launch_axpby3_values(Ctx& c, const BlkIn v[3], const double coef[3], const int* ix, int64_t stride,
                          double gamma, const unsigned char* id, const int* row_of, int64_t nnzb, int b, int64_t n,
                          double* store, int* slot, BlkOut out, const int* live, const int* list);
void launch_block_row_of(Ctx& c, const int* row_ptr, int nb, int64_t nnzb, int* row_of);
void launch_filter_fill(Ctx& c, const int* row_ptr, const int* col, const int* rlab, const int* clab,
                        int mode, const int* new_row_ptr, int nb, int* new_col, int* src);
void launch_transpose_counts(Ctx& c, const int* col, int64_t nnzb, int* counts, const int* live);
// tptr[0..nb]: exclusive prefix sums of the column counts of the first
// *live (else nnzb) entries of col; cursor[0..nb) cleared.  One workgroup,
// for nb with transpose_count_scan_fits(nb).
bool transpose_count_scan_fits(int nb);
void launch_transpose_count_scan(Ctx& c, const int* col, int64_t nnzb, const int* live, int nb, int* tptr,
                                 int* cursor);
void launch_transpose_fill(Ctx& c, const int* row_ptr, const int* col, const int* tptr, int nb,
                           int* cursor, int* tcol, int* tsrc);
void launch_transpose_sort(Ctx& c, const int* tptr, int nb, const int* icol, const int* isrc, int* ocol,
                           int* osrc);
void launch_transpose_blocks(Ctx& c, BlkIn blk, const int* src, int64_t nnzb, int b, double* store, BlkOut out,
                             const int* live);
void launch_segment_sum(Ctx& c, const double* sumsq, const int* row_ptr, const int* rlo, const int* rhi, int nseg,
                        double* out);
void launch_fill_i32(Ctx& c, int* p, int value, int64_t count);
// counts (nrp == null) or fills (nrp given) the blocks of A present in pattern R
void launch_intersect(Ctx& c, const int* ra, const int* ca, const int* rr, const int* cr, int nb, int* counts,
                      const int* nrp, int* ncol, int* src);
void launch_phi_diag(Ctx& c, const int* row_of, const int* col, int64_t nnzb, int b, double* store, BlkOut blk,
                     const int* live);

// spgemm.hip
// Symbolic phase.  opA given as CSR (row ptr, col, value index) of op(A);
// B as CSR of op(B) with value index.  Writes per-row output and product
// counts.
// D (drp, dcol, dblk; nullable) joins the output pattern; the fill pass
// then writes dsrc[e], D's block at output position e (null where D has
// none).
// Operands with holes: `ahole`/`bhole` are their block pointers (null for an
// operand without holes), indexed through aidx/bidx like ablk/bblk; a null
// block takes no part in the product.
// `upper`: only the output blocks (i, j) with j >= i are formed (the upper
// block triangle of a product known to be symmetric).
void launch_symbolic_count(Ctx& c, const int* arp, const int* acol, const int* aidx, const int* brp,
                           const int* bcol, const int* bidx, BlkIn ahole, BlkIn bhole, const int* drp,
                           const int* dcol, int nb, int* cnt_c, int64_t* cnt_p, bool upper = false);
void launch_symbolic_fill(Ctx& c, const int* arp, const int* acol, const int* aidx, const int* brp,
                          const int* bcol, const int* bidx, BlkIn ablk, BlkIn bblk, bool a_holes, bool b_holes,
                          const int* drp, const int* dcol, BlkIn dblk, int nb, const int* crp, const int64_t* prp,
                          int* ccol, int64_t* seg, BlockPair* pairs, BlkOut dsrc, bool upper = false, int row0 = 0,
                          int rows = -1);
// Symbolic phase in one launch when the capacities are known in advance:
// counts, the prefix sums of the row counts (decoupled look-back) and the
// fill.  Writes crp[0..nb]; totals to sizes[0..1]; when a total exceeds its
// capacity the row pointers are all zero and *overflow is raised.  Only for
// nb with symbolic_onepass_fits(nb).
bool symbolic_onepass_fits(int nb);
void launch_symbolic_onepass(Ctx& c, const int* arp, const int* acol, const int* aidx, const int* brp,
                             const int* bcol, const int* bidx, BlkIn ablk, BlkIn bblk, bool a_holes, bool b_holes,
                             const int* drp, const int* dcol, BlkIn dblk, int nb, int64_t cap_c, int64_t cap_p,
                             int* crp, int* ccol, int64_t* seg, BlockPair* pairs, BlkOut dsrc, int64_t* sizes,
                             int* overflow, bool upper = false);
// Fused terms of a product: the output block is alpha sum op(A) op(B)
// + gamma D_e, D_e = dsrc[e] (skipped where null), and its norm is the norm
// of that sum (truncation then applies to the whole block).
// With `drop`, a block whose norm is below `tau` gets a null pointer (the
// product keeps holes instead of being compacted).  When *poison (nullable)
// is set the product is void: no block is computed and workgroup 0 clears
// the row pointers rows[0..nrows].
struct Epilogue {
  double alpha = 1.0;
  double gamma = 0.0;
  BlkIn dsrc = nullptr;
  bool drop = false;
  double tau = 0.0;
  const int* poison = nullptr;
  int* rows = nullptr;
  int nrows = 0;
  // reduced-precision products only (nullable): the output block e is also
  // written transposed in the input precision at lp_store + e b^2 elements,
  // with its pointer (null for a dropped block) in lp_ptr[e]
  void* lp_store = nullptr;
  const void** lp_ptr = nullptr;
  // nullable (with drop): kept blocks take consecutive slots of C (and of
  // lp_store) in the order they finish, counted by this device counter
  // (zero before the launch), so that C holds kept blocks only
  unsigned long long* slots = nullptr;
};

// Thread 0 of an output block's workgroup, once the block's norm is known:
// the slot the block is written to (its own index, or the next free slot of
// a compacted output), or -1 for a dropped block, which is not written.
__device__ inline int64_t output_slot(const Epilogue& epi, int64_t blk, double nrm) {
  if (epi.drop && !(nrm >= epi.tau)) return -1;
  if (epi.slots) return (int64_t)atomicAdd(epi.slots, 1ull);
  return blk;
}

// The numeric kernels' count of output blocks to compute: *live (the grid
// when live is null), or none for a voided product (whose row pointers
// workgroup 0 then clears).
__device__ inline int64_t live_blocks(const int* live, const Epilogue& epi) {
  if (epi.poison && *epi.poison) {
    if (blockIdx.x == 0)
      for (int r = threadIdx.x; r <= epi.nrows; r += blockDim.x) epi.rows[r] = 0;
    return 0;
  }
  return live ? *live : (int64_t)gridDim.x;
}
// Numeric phase: C_blk = sum over its segment of op(A_a) op(B_b), in FP64
// (prec = LIF_FP64) or with FP32 / BF16 inputs and FP32 accumulation.
// `nnzc` is the grid (the output capacity); `live` (device, nullable: all
// nnzc) the number of output blocks actually present, <= nnzc.
// Output block e is written to C + e b^2 (or to the next slot of C, see
// Epilogue::slots), its pointer to Cp[e] and its Frobenius norm to norms[e]
// (nullable).
void launch_numeric(Ctx& c, int prec, bool ta, bool tb, const int64_t* seg, const BlockPair* pairs,
                    int64_t nnzc, const int* live, int b, double* C, BlkOut Cp, double* norms, const Epilogue& epi);
// spgemm_mixed.hip
// Reduced-precision numeric phase: pairs[p].a is op(A)'s block row-major and
// pairs[p].b op(B)'s block transposed, both in the input precision (the
// matrices' copies, Bsr::lp).
void launch_numeric_mixed(Ctx& c, int prec, const int64_t* seg, const BlockPair* pairs, int64_t nnzc,
                          const int* live, int b, double* C, BlkOut Cp, double* norms, const Epilogue& epi);
// Input-precision copies of the first *live of the n blocks blk[e]: block e
// (FP32, or BF16 through FP32, rounded to nearest even; transposed when
// `transposed`) at store + e b^2 elements, ptr[e] its address (null where
// blk[e] is null).
void launch_make_shadow(Ctx& c, int prec, bool transposed, BlkIn blk, int64_t n, const int* live, int b,
                        void* store, const void** ptr);

// chol.hip -- batched leaf inverse Cholesky on packed upper tile grids
void launch_chol_scatter(Ctx& c, const int* row_of, const int* col, BlkIn val, int64_t nnzb, int b,
                         const int* base_of_row, const int* blk0, const int* nbb, const int64_t* tile0, double* U,
                         unsigned char* nz, int* band);
void launch_chol_pad(Ctx& c, int nbase, const int* nbb, const int* rows, const int64_t* tile0, int b, double* M,
                     double value);
void launch_potrf(Ctx& c, int k, int nbase, const int* nbb, const int* blk0, const int64_t* tile0, int b, double* U,
                  double* Z, const unsigned char* nz, int* err);
// `band`: largest j - i over the nonzero tiles (i, j) of S within a leaf;
// the factor's nonzero tiles satisfy j - i <= band as well.
// Step k: the trailing update with the row-k panel of the factor, the
// diagonal factorization of step k + 1 and the V tiles of column k.
void launch_step(Ctx& c, int k, int band, int nbase, int max_nbb, const int* nbb, const int* blk0,
                 const int64_t* tile0, int b, double* U, double* Z, unsigned char* nz, int* err);
// tile columns j0 .. j0 + ncol - 1 of the inverse (those of step j0 + ncol -
// 1 and the steps before it must be done)
void launch_trinv(Ctx& c, int j0, int ncol, int band, int nbase, const int* nbb, const int64_t* tile0, int b,
                  const double* U, double* Z, const unsigned char* nz);

// ---------------------------------------------------------------------------
// Block-sparse operations (ops.cpp): allocate outputs, run the kernels,
// read back the sizes they need.
// ---------------------------------------------------------------------------
struct CsrView {          // CSR of op(A): row ptr, column, index of the stored block
  const int* rp = nullptr;
  const int* col = nullptr;
  const int* idx = nullptr;  // null: identity (block e of A)
  DBuf<int> own_rp, own_col, own_idx;
};

template <typename T>
void h2d(Ctx& c, T* dst, const T* src, size_t count) {
  if (count) LIF_HIP(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, c.stream));
}

// a value array for `blocks` blocks of b*b doubles, from the pool
Store new_store(Ctx& c, int64_t blocks, int b);
// moves A's live blocks into one fresh contiguous store (releasing the
// stores it pointed into); reads the block count back
Bsr compact_values(Ctx& c, Bsr&& A);
Bsr bsr_empty(Ctx& c, int64_t n, int b);
Bsr bsr_from_blocks(Ctx& c, const lif_blocks& in);
// A read-only view of a device block list: row pointers and columns in
// pool memory, block pointers into the caller's value array (no copy).
Bsr bsr_view_blocks(Ctx& c, const lif_blocks& in);
// Checks a block list: shape, sorted unique in-range coordinates, zero
// padding beyond n; optionally a symmetric block pattern (api.cpp).
void validate_blocks(const lif_blocks* B, bool need_symmetric, const char* what);
// The message lif_last_error(NULL) returns on this thread (api.cpp).
void set_thread_error(const std::string& msg);
void bsr_to_blocks(Ctx& c, const Bsr& A, int32_t* brow, int32_t* bcol, double* vals, bool on_device);
DBuf<double> block_norms(Ctx& c, const Bsr& A);
Bsr truncate(Ctx& c, Bsr&& A, const double* norms, double tau);
CsrView transpose_view(Ctx& c, const Bsr& A);
Bsr transpose(Ctx& c, const Bsr& A);
// trunc_tau(alpha op(A) op(B) [+ gamma D]): the optional term D is added
// block by block before the truncation.  With `keep_holes` the dropped
// blocks stay in the pattern with null pointers (Bsr::holes) instead of
// being compacted away, for a result that only products and sums read.
// Records `out` as the result of one task that depends on the matrices in
// `in` (null entries ignored): its chain is one longer than the longest of
// theirs (among equally long ones, the one with most products).
void task_after(Ctx& c, Bsr& out, bool product, std::initializer_list<const Bsr*> in);
// With prec FP32 / BF16 the operands are read from their input-precision
// copies (made here when missing); `out_lp`: with keep_holes, the result
// also gets its transposed copy ([1]) in that precision, for a later
// reduced-precision product that takes it as right operand.
// `upper`: only the output blocks (i, j) with j >= i (the upper block
// triangle, for a product whose caller uses only that part).
Bsr spgemm(Ctx& c, const Bsr& A, bool ta, const Bsr& B, bool tb, double tau, int prec = LIF_FP64,
           double alpha = 1.0, const Bsr* D = nullptr, double gamma = 0.0, bool keep_holes = false,
           bool out_lp = false, bool upper = false);
// makes A.lp[layout] hold A's blocks in precision prec (no-op when it does)
void ensure_shadow(Ctx& c, const Bsr& A, int prec, int layout);
// alpha A + beta B + gamma I on the block rows with diag_on set (A or B may be null)
Bsr axpby(Ctx& c, double alpha, const Bsr* A, double beta, const Bsr* B, double gamma,
          const unsigned char* diag_on);
// alpha A + beta B + kappa C in one pass (any may be null)
Bsr axpby3(Ctx& c, double alpha, const Bsr* A, double beta, const Bsr* B, double kappa, const Bsr* C);
Bsr filter(Ctx& c, const Bsr& A, const int* rlab, const int* clab, int mode);
double gershgorin(Ctx& c, const Bsr& A);
std::vector<double> node_sumsq(Ctx& c, const Bsr& A, const int* rlo, const int* rhi, int nseg,
                               const std::vector<Ctx::Read>& extra = {});
Bsr copy(Ctx& c, const Bsr& A);
// exact block count (reads it from the device when only the device knows it)
int64_t exact_nnzb(Ctx& c, const Bsr& A);
// blocks of A that also occur in R's pattern
Bsr intersect(Ctx& c, const Bsr& A, const Bsr& R);
// upper block triangle of W with the diagonal blocks' upper triangles and
// halved diagonals (the mask of the inverse-Cholesky adjoint)
Bsr phi_upper(Ctx& c, const Bsr& W);

}  // namespace lif
