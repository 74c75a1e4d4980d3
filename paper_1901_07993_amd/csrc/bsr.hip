// Block-CSR utility kernels: row pointers, block norms, truncation and
// compaction (Sec. 5: blocks with Frobenius norm < tau are removed), pattern
// union with scaled sums (matrix addition / scaling, identity terms),
// filters that cut level- and coupling-parts out of a matrix, transposition,
// the Gershgorin bound (Sec. 2.2) and segmented norm sums.
//
// Value blocks are reached through per-matrix pointer arrays and are written
// once: truncation, filters and copies move 8-byte pointers, and a sum whose
// block comes from one operand unscaled points at that operand's block.
// Passes that do touch values handle one block per workgroup with coalesced
// 16-byte accesses; index work runs one thread per block row or block.
#include "block_scan.h"
#include "lookback.h"
#include "common.h"
#include "tile_mma.h"

namespace lif {

namespace {

constexpr int kWG = 256;

// A b x b block handled by 256 threads: each thread holds V2 consecutive
// double pairs.  The loads of a block are all issued before the first use
// (unrolled over V2), so a block costs one memory latency, not V2 of them.
template <int B>
struct Blk {
  static constexpr int V2 = B * B / 2 / kWG;
};

template <int B>
__device__ __attribute__((always_inline)) inline void blk_load(const double* __restrict__ p, v2d (&r)[Blk<B>::V2]) {
  const auto* q = gptr(reinterpret_cast<const v2d*>(p));
#pragma unroll
  for (int v = 0; v < Blk<B>::V2; ++v) r[v] = q[threadIdx.x + v * kWG];
}

template <int B>
__device__ __attribute__((always_inline)) inline void blk_store(double* __restrict__ p, const v2d (&r)[Blk<B>::V2]) {
  v2d* q = reinterpret_cast<v2d*>(p);
#pragma unroll
  for (int v = 0; v < Blk<B>::V2; ++v) q[threadIdx.x + v * kWG] = r[v];
}

// element index (row-major in the block) of the first double of pair v
template <int B>
__device__ __attribute__((always_inline)) inline int blk_elem(int v) {
  return 2 * (threadIdx.x + v * kWG);
}

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Fixed-order block sum of one double per thread (256 threads): wave sums,
// then the 4 wave totals added in order by thread 0.  Deterministic.
__device__ inline double block_sum_256(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
  return r;
}

__global__ void k_row_ptr_from_rows(const int* __restrict__ brow, int64_t nnzb, int nb, int* __restrict__ rp) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e > nnzb) return;
  int prev = (e == 0) ? -1 : brow[e - 1];
  int cur = (e == nnzb) ? nb : brow[e];
  for (int r = prev + 1; r <= cur; ++r) rp[r] = (int)e;
}

template <int B>
__global__ __launch_bounds__(kWG) void k_block_sumsq(BlkIn blk, int64_t nnzb, double* __restrict__ out,
                                                     int take_sqrt, const int* __restrict__ live) {
  __shared__ double sh[4];
  const int64_t e = blockIdx.x;
  if (live && e >= *live) return;
  v2d r[Blk<B>::V2];
  blk_load<B>(blk[e], r);
  double s = 0.0;
#pragma unroll
  for (int v = 0; v < Blk<B>::V2; ++v) s += r[v].x * r[v].x + r[v].y * r[v].y;
  double t = block_sum_256(s, sh);
  if (threadIdx.x == 0) out[e] = take_sqrt ? sqrt(t) : t;
}

__global__ void k_gather_ptrs(BlkIn blk, const int* __restrict__ src, int64_t nnzb, BlkOut out,
                              const int* __restrict__ live) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnzb || (live && e >= *live)) return;
  out[e] = blk[src[e]];
}

// out[e] = base + e bb: the pointers of a contiguous value array
__global__ void k_fill_ptrs(BlkOut out, const double* base, int bb, int64_t count) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) out[e] = base + e * bb;
}

// contiguous copy of the blocks (block e to out + e bb)
template <int B>
__global__ __launch_bounds__(kWG) void k_gather_values(BlkIn blk, double* __restrict__ out,
                                                       const int* __restrict__ live) {
  const int64_t e = blockIdx.x;
  if (live && e >= *live) return;
  v2d r[Blk<B>::V2];
  blk_load<B>(blk[e], r);
  blk_store<B>(out + e * B * B, r);
}

// Gershgorin: row_max[i] = max over the b scalar rows of block row i of
// sum_j |S_rj|.  One workgroup per block row; each wave takes scalar rows
// w, w+4, ... and reads them 64 doubles at a time.
__global__ __launch_bounds__(kWG) void k_gershgorin(const int* __restrict__ rp, BlkIn blk, int b,
                                                    double* __restrict__ row_max) {
  __shared__ double sh[4];
  const int i = blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double best = 0.0;
  for (int r = w; r < b; r += 4) {
    double s = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
      const auto* row = gptr(blk[e] + (int64_t)r * b);
      for (int cc = lane; cc < b; cc += 64) s += fabs(row[cc]);
    }
    s = wave_sum(s);
    best = fmax(best, s);
  }
  if (lane == 0) sh[w] = best;
  __syncthreads();
  if (threadIdx.x == 0) row_max[i] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

__global__ __launch_bounds__(1024) void k_max_reduce(const double* __restrict__ in, int count, double* __restrict__ out) {
  __shared__ double sh[16];
  double m = 0.0;
  for (int i = threadIdx.x; i < count; i += 1024) m = fmax(m, in[i]);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int k = 0; k < 16; ++k) r = fmax(r, sh[k]);
    out[0] = r;
  }
}

// Union of the sorted column lists of up to three operands' row i, plus
// column i when diag_on[i] is set.  Absent operands have null pointers; an
// operand with holes gives its block pointers in `hole`, and its null
// blocks are skipped.
struct Src3 {
  const int* rp[3];
  const int* col[3];
  BlkIn hole[3];
};

__device__ inline void skip_holes(const Src3& S, int t, int& p, int e) {
  if (S.hole[t])
    while (p < e && !S.hole[t][p]) ++p;
}

__device__ inline int union_row(const Src3& S, const unsigned char* diag_on, int i, int* cc, int* ix,
                                int64_t stride, unsigned char* id, int* rowof) {
  int p[3], e[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    p[t] = S.rp[t] ? S.rp[t][i] : 0;
    e[t] = S.rp[t] ? S.rp[t][i + 1] : 0;
    skip_holes(S, t, p[t], e[t]);
  }
  bool dg = diag_on && diag_on[i];
  int o = 0;
  while (p[0] < e[0] || p[1] < e[1] || p[2] < e[2] || dg) {
    int x = dg ? i : INT_MAX;
#pragma unroll
    for (int t = 0; t < 3; ++t)
      if (p[t] < e[t]) x = min(x, S.col[t][p[t]]);
    if (cc) {
      cc[o] = x;
      id[o] = (dg && x == i) ? 1 : 0;
      rowof[o] = i;
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const bool hit = p[t] < e[t] && S.col[t][p[t]] == x;
      if (cc) ix[t * stride + o] = hit ? p[t] : -1;
      if (hit) {
        ++p[t];
        skip_holes(S, t, p[t], e[t]);
      }
    }
    if (dg && x == i) dg = false;
    ++o;
  }
  return o;
}

// also clears the slot counter of the values pass that follows
__global__ void k_union_counts(Src3 S, const unsigned char* diag_on, int nb, int* counts, int* slot) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot && i == 0) *slot = 0;
  if (i >= nb) return;
  counts[i] = union_row(S, diag_on, i, nullptr, nullptr, 0, nullptr, nullptr);
}

// ix holds three index arrays of length stride (one per source), -1 = absent
__global__ void k_union_fill(Src3 S, const unsigned char* diag_on, const int* rc, int nb, int* cc, int* ix,
                             int64_t stride, unsigned char* id, int* rowof) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  int o = rc[i];
  union_row(S, diag_on, i, cc + o, ix + o, stride, id + o, rowof + o);
}

// The same union with one wave per block row: the operands' columns are
// marked in LDS bitmaps (one per operand; the index of each marked column in
// its operand kept in an nb-long LDS map), the union is their OR, and the
// output positions come from popcounts of the OR's words -- the row's
// entries are handled in parallel instead of merged one by one.
constexpr int kUR = 64;

inline size_t union_rows_lds(int nb, bool fill) {
  const size_t nwords = (size_t)(nb + 31) / 32;
  return fill ? (4 * nwords + 3 * (size_t)nb) * 4 : 3 * nwords * 4;
}

// One-pass unions also sort the output blocks into those taken unchanged
// from one operand (a unit coefficient, no identity term: the union writes
// the operand's block pointer to out) and those that need new values,
// listed in list[0..*ncomp) for the values pass; the list is in row order
// (each row's part placed by the same look-back as its output positions).
struct UnionList {
  BlkIn val[3];
  bool unit[3];
  BlkOut out;
  int* list;
  int* ncomp;
};

// Whether output column j (bit `bit` of word w) of the row needs new
// values; *tsrc is the operand holding it when it has a single one.
__device__ inline bool union_needs_value(const Src3& S, const UnionList& L, const unsigned* bm, int nwords, int w,
                                         int bit, bool dgj, int* tsrc) {
  int present = 0, t1 = 0;
#pragma unroll
  for (int t = 0; t < 3; ++t)
    if (S.rp[t] && ((bm[t * nwords + w] >> bit) & 1u)) {
      ++present;
      t1 = t;
    }
  *tsrc = t1;
  return dgj || present != 1 || !L.unit[t1];
}

// MODE 0: counts[i]; 1: fill at the row pointers rc; 2: one pass -- the
// row pointers are the prefix sums of the counts over the lower rows,
// obtained by look-back (lookback.h) and written to rc by each row.  Modes 0
// and 2 also zero *slot.
template <int MODE>
__global__ __launch_bounds__(kUR) void k_union_rows(Src3 S, const unsigned char* __restrict__ diag_on, int nb,
                                                    int* __restrict__ counts, int* __restrict__ slot,
                                                    int* __restrict__ rc, int* __restrict__ cc,
                                                    int* __restrict__ ix, int64_t stride,
                                                    unsigned char* __restrict__ id, int* __restrict__ rowof,
                                                    Ctx::LbWords lbw, UnionList L) {
  constexpr bool FILL = MODE != 0;
  extern __shared__ unsigned smem[];
  __shared__ int scan_tmp[1], scan_tmp2[1];
  const int i = blockIdx.x;
  const int nwords = (nb + 31) >> 5;
  unsigned* bm = smem;                              // [3][nwords]
  int* c2i = reinterpret_cast<int*>(smem + 4 * nwords);  // [3][nb] (fill)
  if (MODE != 1 && slot && i == 0 && threadIdx.x == 0) *slot = 0;
  for (int w = threadIdx.x; w < 3 * nwords; w += kUR) bm[w] = 0u;
  __syncthreads();
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    if (!S.rp[t]) continue;
    const int hi = S.rp[t][i + 1];
    for (int p = S.rp[t][i] + threadIdx.x; p < hi; p += kUR) {
      if (S.hole[t] && !S.hole[t][p]) continue;
      const int j = S.col[t][p];
      atomicOr(&bm[t * nwords + (j >> 5)], 1u << (j & 31));
      if (FILL) c2i[t * nb + j] = p;
    }
  }
  const bool dg = diag_on && diag_on[i];
  __syncthreads();
  const unsigned dbit = 1u << (i & 31);
  auto word = [&](int w) {
    unsigned u = bm[w] | bm[nwords + w] | bm[2 * nwords + w];
    if (dg && (i >> 5) == w) u |= dbit;
    return u;
  };
  const int chunk = (nwords + kUR - 1) / kUR;  // contiguous words per lane
  const int w0 = min(nwords, (int)threadIdx.x * chunk), w1 = min(nwords, w0 + chunk);
  int s = 0;
  for (int w = w0; w < w1; ++w) s += __popc(word(w));
  if (!FILL) {
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (threadIdx.x == 0) counts[i] = s;
    return;
  }
  int total;
  int r = block_exclusive_scan<int, kUR>(s, scan_tmp, &total);
  int q = 0;  // position in the list of blocks that need values (MODE 2)
  if (MODE == 2) {  // one wave: the whole workgroup takes part in the look-back
    int nc = 0;
    for (int w = w0; w < w1; ++w) {
      unsigned bits = word(w);
      while (bits) {
        const int bit = __ffs(bits) - 1;
        int tsrc;
        nc += union_needs_value(S, L, bm, nwords, w, bit, dg && (w << 5) + bit == i, &tsrc) ? 1 : 0;
        bits &= bits - 1;
      }
    }
    int nctot;
    q = block_exclusive_scan<int, kUR>(nc, scan_tmp2, &nctot);
    unsigned long long ea = 0, eb = 0;
    const bool ok = lb_exclusive2(lbw.ra, lbw.rb, lbw.ga, lbw.gb, i, nb, lbw.epoch, (unsigned long long)total,
                                  (unsigned long long)nctot, &ea, &eb);
    // a union's size is bounded by its operands', so no capacity can be
    // short; a look-back that gave up leaves the prefix at 0 (in bounds,
    // wrong) and raises the flag the host checks
    if (!ok && threadIdx.x == 0) atomicExch(lbw.fail, 1);
    const int base = ok ? (int)ea : 0, qbase = ok ? (int)eb : 0;
    if (threadIdx.x == 0) {
      rc[i] = base;
      if (i == nb - 1) {
        rc[nb] = base + total;
        *L.ncomp = qbase + nctot;
      }
    }
    r += base;
    q += qbase;
  } else {
    r += rc[i];
  }
  for (int w = w0; w < w1; ++w) {
    unsigned bits = word(w);
    while (bits) {
      const int bit = __ffs(bits) - 1;
      const int j = (w << 5) + bit;
      cc[r] = j;
      id[r] = (dg && j == i) ? 1 : 0;
      rowof[r] = i;
#pragma unroll
      for (int t = 0; t < 3; ++t)
        ix[t * stride + r] = (S.rp[t] && ((bm[t * nwords + w] >> bit) & 1u)) ? c2i[t * nb + j] : -1;
      if (MODE == 2) {
        int tsrc;
        if (union_needs_value(S, L, bm, nwords, w, bit, dg && j == i, &tsrc))
          L.list[q++] = r;
        else
          L.out[r] = L.val[tsrc][c2i[tsrc * nb + j]];
      }
      ++r;
      bits &= bits - 1;
    }
  }
}

struct Val3 {
  BlkIn v[3];
  double coef[3];
};

// out = sum_t coef_t src_t[ix_t] + gamma I (diagonal entries of real rows only)
// One output block per workgroup.  A block taken unscaled from a single
// operand, with no identity term, is not copied: its pointer is reused.
// Every other block is computed into the next free slot of `store` (slots
// are handed out by an atomic counter; where a block lands does not change
// its value).
// LIST: one workgroup per entry w of list (the blocks that need values),
// *live entries, output block e = list[w], store slot w.
template <int B, bool LIST>
__global__ __launch_bounds__(kWG) void k_axpby_values(Val3 V, const int* __restrict__ ix, int64_t stride,
                                                      double gamma, const unsigned char* __restrict__ id,
                                                      const int* __restrict__ row_of, int64_t n,
                                                      double* __restrict__ store, int* __restrict__ slot,
                                                      BlkOut out, const int* __restrict__ live,
                                                      const int* __restrict__ list) {
  __shared__ int my_slot;
  if (live && (int64_t)blockIdx.x >= *live) return;
  const int64_t e = LIST ? list[blockIdx.x] : blockIdx.x;
  const double* src[3];
  double cf[3];
  int ns = 0;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const int x = V.v[t] ? ix[t * stride + e] : -1;
    if (x >= 0) {
      src[ns] = V.v[t][x];
      cf[ns] = V.coef[t];
      ++ns;
    }
  }
  const bool dg = id[e] != 0;
  if (!LIST && ns == 1 && cf[0] == 1.0 && !dg) {
    if (threadIdx.x == 0) out[e] = src[0];
    return;
  }
  if (LIST) {
    if (threadIdx.x == 0) my_slot = (int)blockIdx.x;
  } else if (threadIdx.x == 0) {
    my_slot = atomicAdd(slot, 1);
  }
  // all operand loads in flight before the first use; the sum keeps the
  // operand order: ((0 + c0 v0) + c1 v1) + c2 v2
  v2d r[3][Blk<B>::V2];
#pragma unroll
  for (int t = 0; t < 3; ++t)
    if (t < ns) blk_load<B>(src[t], r[t]);
  v2d acc[Blk<B>::V2];
#pragma unroll
  for (int v = 0; v < Blk<B>::V2; ++v) {
    acc[v] = v2d{0.0, 0.0};
#pragma unroll
    for (int t = 0; t < 3; ++t)
      if (t < ns) {
        acc[v].x += cf[t] * r[t][v].x;
        acc[v].y += cf[t] * r[t][v].y;
      }
  }
  if (dg) {
    const int64_t row0 = (int64_t)row_of[e] * B;
#pragma unroll
    for (int v = 0; v < Blk<B>::V2; ++v) {
      const int lin = blk_elem<B>(v);
      const int rr = lin / B, c0 = lin % B;
      if (row0 + rr < n) {
        if (c0 == rr) acc[v].x += gamma;
        if (c0 + 1 == rr) acc[v].y += gamma;
      }
    }
  }
  __syncthreads();
  double* dst = store + (int64_t)my_slot * B * B;
  blk_store<B>(dst, acc);
  if (threadIdx.x == 0) out[e] = dst;
}

__global__ void k_block_row_of(const int* __restrict__ rp, int nb, int* __restrict__ row_of) {
  int i = blockIdx.x;
  for (int e = rp[i] + threadIdx.x; e < rp[i + 1]; e += blockDim.x) row_of[e] = i;
}

// Filter predicates on per-block-row labels of the row (rlab) and of the
// column (clab):
//   mode 0: rlab[i] >= 0 && rlab[i] == clab[j]            (same group)
//   mode 1: rlab[i] >= 0, rlab[i] even, clab[j] == rlab[i] + 1
//           (labels 2 g + side: leading part A to trailing part C of group g)
//   mode 2: rlab[i] >= 0                                   (rows of active groups)
//   mode 3: rlab[i] >= 0 && clab[j] >= rlab[i]             (upper block triangle
//           when the labels are the block indices)
__device__ inline bool keep_pred(int mode, int li, int lj) {
  if (li < 0) return false;
  if (mode == 0) return li == lj;
  if (mode == 1) return ((li & 1) == 0) && lj == li + 1;
  if (mode == 3) return lj >= li;
  return true;
}

__global__ void k_filter_fill(const int* __restrict__ rp, const int* __restrict__ col, const int* __restrict__ rlab,
                              const int* __restrict__ clab, int mode, const int* __restrict__ nrp, int nb,
                              int* __restrict__ ncol, int* __restrict__ src) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  int li = rlab[i];
  if (li < 0) return;
  int o = nrp[i];
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    if (keep_pred(mode, li, clab[col[e]])) {
      ncol[o] = col[e];
      src[o] = e;
      ++o;
    }
  }
}

__global__ void k_transpose_counts(const int* __restrict__ col, int64_t nnzb, int* __restrict__ counts,
                                   const int* __restrict__ live) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t lim = live ? min(nnzb, (int64_t)*live) : nnzb;
  if (e < lim) atomicAdd(&counts[col[e]], 1);
}

// The column counts of a pattern, their exclusive prefix sums (the row
// pointers of the transposed pattern) and a cleared cursor per column for
// the fill, in one workgroup: the counts are LDS atomics, the scan runs over
// contiguous runs of columns per thread.  LDS: nb counters.
constexpr int kTC = 1024;
__global__ __launch_bounds__(kTC) void k_transpose_count_scan(const int* __restrict__ col, int64_t nnzb,
                                                              const int* __restrict__ live, int nb,
                                                              int* __restrict__ tptr, int* __restrict__ cursor) {
  extern __shared__ int cnt[];
  __shared__ int sh[kTC / 64];
  for (int j = threadIdx.x; j < nb; j += kTC) cnt[j] = 0;
  __syncthreads();
  const int64_t lim = live ? min(nnzb, (int64_t)*live) : nnzb;
  for (int64_t e = threadIdx.x; e < lim; e += kTC) atomicAdd(&cnt[col[e]], 1);
  __syncthreads();
  const int chunk = (nb + kTC - 1) / kTC;
  const int lo = min(nb, (int)threadIdx.x * chunk), hi = min(nb, lo + chunk);
  int s = 0;
  for (int j = lo; j < hi; ++j) s += cnt[j];
  int total;
  int run = block_exclusive_scan<int, kTC>(s, sh, &total);
  for (int j = lo; j < hi; ++j) {
    tptr[j] = run;
    run += cnt[j];
    cursor[j] = 0;
  }
  if (threadIdx.x == 0) tptr[nb] = total;
}

__global__ void k_transpose_fill(const int* __restrict__ rp, const int* __restrict__ col, const int* __restrict__ tptr,
                                 int nb, int* __restrict__ cursor, int* __restrict__ tcol, int* __restrict__ tsrc) {
  int i = blockIdx.x;
  for (int e = rp[i] + threadIdx.x; e < rp[i + 1]; e += blockDim.x) {
    int j = col[e];
    int pos = tptr[j] + atomicAdd(&cursor[j], 1);
    tcol[pos] = i;
    tsrc[pos] = e;
  }
}

// Sort each transposed row by its (distinct) column keys: every element's
// rank is the number of smaller keys in its segment, and it is written to
// that rank of the output arrays.  Keys are staged in LDS when the segment
// fits (4096 entries), else read from HBM.  Out of place, so any segment
// length is handled.
constexpr int kSortLds = 4096;
__global__ __launch_bounds__(kWG) void k_transpose_sort(const int* __restrict__ tptr, const int* __restrict__ icol,
                                                        const int* __restrict__ isrc, int* __restrict__ ocol,
                                                        int* __restrict__ osrc) {
  __shared__ int key[kSortLds];
  const int j = blockIdx.x;
  const int lo = tptr[j], len = tptr[j + 1] - tptr[j];
  const bool staged = len <= kSortLds;
  if (staged) {
    for (int t = threadIdx.x; t < len; t += kWG) key[t] = icol[lo + t];
    __syncthreads();
  }
  const int* keys = staged ? key : icol + lo;
  for (int t = threadIdx.x; t < len; t += kWG) {
    const int k = keys[t];
    int r = 0;
    for (int u = 0; u < len; ++u) r += (keys[u] < k) ? 1 : 0;
    ocol[lo + r] = k;
    osrc[lo + r] = isrc[lo + t];
  }
}

template <int B>
__global__ __launch_bounds__(kWG) void k_transpose_blocks(BlkIn blk, const int* __restrict__ src,
                                                          double* __restrict__ store, BlkOut out,
                                                          const int* __restrict__ live) {
  __shared__ double t[B * (B + 1)];
  const int64_t e = blockIdx.x;
  if (live && e >= *live) return;
  v2d r[Blk<B>::V2];
  blk_load<B>(blk[src[e]], r);
#pragma unroll
  for (int v = 0; v < Blk<B>::V2; ++v) {
    const int q = blk_elem<B>(v), rr = q / B, cc = q % B;
    t[cc * (B + 1) + rr] = r[v].x;
    t[(cc + 1) * (B + 1) + rr] = r[v].y;
  }
  __syncthreads();
#pragma unroll
  for (int v = 0; v < Blk<B>::V2; ++v) {
    const int q = blk_elem<B>(v), rr = q / B, cc = q % B;
    r[v] = v2d{t[rr * (B + 1) + cc], t[rr * (B + 1) + cc + 1]};
  }
  double* d = store + e * B * B;
  blk_store<B>(d, r);
  if (threadIdx.x == 0) out[e] = d;
}

// out[s] = sum of sumsq[e] over the blocks of block rows [rlo[s], rhi[s])
__global__ __launch_bounds__(kWG) void k_segment_sum(const double* __restrict__ sumsq, const int* __restrict__ rp,
                                                     const int* __restrict__ rlo, const int* __restrict__ rhi,
                                                     double* __restrict__ out) {
  __shared__ double sh[4];
  const int s = blockIdx.x;
  const int lo = rp[rlo[s]], hi = rp[rhi[s]];
  double v = 0.0;
  for (int e = lo + threadIdx.x; e < hi; e += kWG) v += sumsq[e];
  double r = block_sum_256(v, sh);
  if (threadIdx.x == 0) out[s] = r;
}

// Blocks of A whose coordinates also occur in the reference pattern R.
__global__ void k_intersect_counts(const int* __restrict__ ra, const int* __restrict__ ca, const int* __restrict__ rr,
                                   const int* __restrict__ cr, int nb, int* __restrict__ counts,
                                   const int* __restrict__ nrp, int* __restrict__ ncol, int* __restrict__ src) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  int pa = ra[i], ea = ra[i + 1], pr = rr[i], er = rr[i + 1];
  int o = nrp ? nrp[i] : 0, cnt = 0;
  while (pa < ea && pr < er) {
    const int xa = ca[pa], xr = cr[pr];
    if (xa == xr) {
      if (nrp) {
        ncol[o] = xa;
        src[o] = pa;
        ++o;
      }
      ++cnt;
      ++pa;
      ++pr;
    } else if (xa < xr) {
      ++pa;
    } else {
      ++pr;
    }
  }
  if (!nrp) counts[i] = cnt;
}

// Inverse-Cholesky adjoint mask on block row/col coordinates: diagonal
// blocks keep their upper triangle with the diagonal halved (written to slot
// `row` of `store`, the pointer redirected there); other blocks are left as
// they are (the caller keeps only blocks with col >= row).
template <int B>
__global__ __launch_bounds__(kWG) void k_phi_diag(const int* __restrict__ row_of, const int* __restrict__ col,
                                                  double* __restrict__ store, BlkOut blk,
                                                  const int* __restrict__ live) {
  const int64_t e = blockIdx.x;
  if (live && e >= *live) return;
  const int i = row_of[e];
  if (i != col[e]) return;
  v2d r[Blk<B>::V2];
  blk_load<B>(blk[e], r);
#pragma unroll
  for (int v = 0; v < Blk<B>::V2; ++v) {
    const int q = blk_elem<B>(v), rr = q / B, cc = q % B;
    r[v].x = (cc < rr) ? 0.0 : (cc == rr ? 0.5 * r[v].x : r[v].x);
    r[v].y = (cc + 1 < rr) ? 0.0 : (cc + 1 == rr ? 0.5 * r[v].y : r[v].y);
  }
  double* d = store + (int64_t)i * B * B;
  blk_store<B>(d, r);
  __syncthreads();  // every read of the old block done before the pointer moves
  if (threadIdx.x == 0) blk[e] = d;
}

// ---------------------------------------------------------------------------
// Per-row counts and their exclusive prefix sum in one workgroup: each thread
// takes a contiguous run of rows, counts them, the run totals are scanned in
// LDS, then each thread counts its rows again while writing the row pointers.
// One launch instead of a count kernel and a scan kernel.
// ---------------------------------------------------------------------------
constexpr int kCS = 1024;

template <class Count>
__global__ __launch_bounds__(kCS) void k_count_scan(Count cnt, int nb, int* __restrict__ rp) {
  __shared__ int sh[kCS / 64];
  const int t = threadIdx.x;
  const int chunk = (nb + kCS - 1) / kCS;
  const int lo = min(nb, t * chunk), hi = min(nb, lo + chunk);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += cnt(i);
  int total;
  int run = block_exclusive_scan<int, kCS>(s, sh, &total);
  for (int i = lo; i < hi; ++i) {
    rp[i] = run;
    run += cnt(i);
  }
  if (t == 0) rp[nb] = total;
}

struct KeepCount {
  const int* rp;
  const double* norms;
  double tau;
  __device__ int operator()(int i) const {
    int c = 0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) c += (norms[e] >= tau) ? 1 : 0;
    return c;
  }
};

struct FilterCount {
  const int* rp;
  const int* col;
  const int* rlab;
  const int* clab;
  int mode;
  __device__ int operator()(int i) const {
    const int li = rlab[i];
    if (li < 0) return 0;
    int c = 0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) c += keep_pred(mode, li, clab[col[e]]) ? 1 : 0;
    return c;
  }
};

struct IntersectCount {
  const int* ra;
  const int* ca;
  const int* rr;
  const int* cr;
  __device__ int operator()(int i) const {
    int pa = ra[i], ea = ra[i + 1], pr = rr[i], er = rr[i + 1], c = 0;
    while (pa < ea && pr < er) {
      const int xa = ca[pa], xr = cr[pr];
      if (xa == xr) {
        ++c;
        ++pa;
        ++pr;
      } else if (xa < xr) {
        ++pa;
      } else {
        ++pr;
      }
    }
    return c;
  }
};

// Truncation compaction, one thread per block of the untruncated matrix: a
// kept block finds its row (binary search in the row pointers) and its rank
// among the kept blocks before it in that row; its column and value pointer
// move there.
__global__ void k_compact_gather(const int* __restrict__ rp, int nb, const int* __restrict__ col,
                                 const double* __restrict__ norms, double tau, const int* __restrict__ nrp,
                                 BlkIn blk, int64_t nnzb, int* __restrict__ ncol, BlkOut nblk) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnzb || e >= rp[nb] || !(norms[e] >= tau)) return;
  int lo = 0, hi = nb;  // largest row with rp[row] <= e
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (rp[mid] <= e) lo = mid;
    else hi = mid;
  }
  int rank = 0;
  for (int64_t f = rp[lo]; f < e; ++f) rank += (norms[f] >= tau) ? 1 : 0;
  const int dst = nrp[lo] + rank;
  ncol[dst] = col[e];
  nblk[dst] = blk[e];
}

__global__ void k_fill_i32(int* p, int value, int64_t count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

inline unsigned grid1(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

#define LIF_LAUNCH(...)                   \
  do {                                    \
    hipLaunchKernelGGL(__VA_ARGS__);      \
    LIF_HIP(hipGetLastError());           \
  } while (0)

void launch_row_ptr_from_rows(Ctx& c, const int* brow, int64_t nnzb, int nb, int* row_ptr) {
  LIF_LAUNCH(k_row_ptr_from_rows, dim3(grid1(nnzb + 1, 256)), dim3(256), 0, c.stream, brow, nnzb, nb, row_ptr);
}

void launch_block_sumsq(Ctx& c, BlkIn blk, int64_t nnzb, int b, double* out, bool take_sqrt, const int* live) {
  if (nnzb == 0) return;
  if (b == 64)
    LIF_LAUNCH(k_block_sumsq<64>, dim3((unsigned)nnzb), dim3(kWG), 0, c.stream, blk, nnzb, out, take_sqrt ? 1 : 0,
               live);
  else
    LIF_LAUNCH(k_block_sumsq<32>, dim3((unsigned)nnzb), dim3(kWG), 0, c.stream, blk, nnzb, out, take_sqrt ? 1 : 0,
               live);
}

void launch_gather_ptrs(Ctx& c, BlkIn blk, const int* src, int64_t nnzb, BlkOut out, const int* live) {
  if (nnzb == 0) return;
  LIF_LAUNCH(k_gather_ptrs, dim3(grid1(nnzb, 256)), dim3(256), 0, c.stream, blk, src, nnzb, out, live);
}

void launch_fill_ptrs(Ctx& c, BlkOut out, const double* base, int b, int64_t count) {
  if (count == 0) return;
  LIF_LAUNCH(k_fill_ptrs, dim3(grid1(count, 256)), dim3(256), 0, c.stream, out, base, b * b, count);
}

void launch_gather_values(Ctx& c, BlkIn blk, int64_t nnzb, int b, double* out, const int* live) {
  if (nnzb == 0) return;
  if (b == 64)
    LIF_LAUNCH(k_gather_values<64>, dim3((unsigned)nnzb), dim3(kWG), 0, c.stream, blk, out, live);
  else
    LIF_LAUNCH(k_gather_values<32>, dim3((unsigned)nnzb), dim3(kWG), 0, c.stream, blk, out, live);
}

void launch_gershgorin(Ctx& c, const int* row_ptr, BlkIn blk, int nb, int b, double* row_max) {
  LIF_LAUNCH(k_gershgorin, dim3(nb), dim3(kWG), 0, c.stream, row_ptr, blk, b, row_max);
}

void launch_max_reduce(Ctx& c, const double* in, int count, double* out) {
  LIF_LAUNCH(k_max_reduce, dim3(1), dim3(1024), 0, c.stream, in, count, out);
}

// the row-parallel union while its LDS stays within the default limit
// (block rows nb up to about 4000); the per-thread merge above that
constexpr size_t kUnionRowsLds = 48 * 1024;

void launch_union3(Ctx& c, const int* const rp[3], const int* const col[3], const BlkIn hole[3],
                   const unsigned char* diag_on, int nb, int* counts, int* slot) {
  Src3 S;
  for (int t = 0; t < 3; ++t) {
    S.rp[t] = rp[t];
    S.col[t] = col[t];
    S.hole[t] = hole[t];
  }
  if (union_rows_lds(nb, true) <= kUnionRowsLds) {
    LIF_LAUNCH(k_union_rows<0>, dim3(nb), dim3(kUR), union_rows_lds(nb, false), c.stream, S, diag_on, nb, counts,
               slot, nullptr, nullptr, nullptr, 0, nullptr, nullptr, Ctx::LbWords{}, UnionList{});
    return;
  }
  LIF_LAUNCH(k_union_counts, dim3(grid1(nb, 128)), dim3(128), 0, c.stream, S, diag_on, nb, counts, slot);
}

void launch_union3_fill(Ctx& c, const int* const rp[3], const int* const col[3], const BlkIn hole[3],
                        const unsigned char* diag_on, const int* rc, int nb, int* cc, int* ix, int64_t stride,
                        unsigned char* id, int* rowof) {
  Src3 S;
  for (int t = 0; t < 3; ++t) {
    S.rp[t] = rp[t];
    S.col[t] = col[t];
    S.hole[t] = hole[t];
  }
  if (union_rows_lds(nb, true) <= kUnionRowsLds) {
    LIF_LAUNCH(k_union_rows<1>, dim3(nb), dim3(kUR), union_rows_lds(nb, true), c.stream, S, diag_on, nb, nullptr,
               nullptr, const_cast<int*>(rc), cc, ix, stride, id, rowof, Ctx::LbWords{}, UnionList{});
    return;
  }
  LIF_LAUNCH(k_union_fill, dim3(grid1(nb, 128)), dim3(128), 0, c.stream, S, diag_on, rc, nb, cc, ix, stride, id,
             rowof);
}

bool union_onepass_fits(int nb) { return union_rows_lds(nb, true) <= kUnionRowsLds; }

void launch_union3_onepass(Ctx& c, const int* const rp[3], const int* const col[3], const BlkIn hole[3],
                           const BlkIn val[3], const double coef[3], const unsigned char* diag_on, int* rc, int nb,
                           int* cc, int* ix, int64_t stride, unsigned char* id, int* rowof, BlkOut out, int* list,
                           int* ncomp) {
  Src3 S;
  UnionList L;
  for (int t = 0; t < 3; ++t) {
    S.rp[t] = rp[t];
    S.col[t] = col[t];
    S.hole[t] = hole[t];
    L.val[t] = val[t];
    L.unit[t] = coef[t] == 1.0;
  }
  L.out = out;
  L.list = list;
  L.ncomp = ncomp;
  const Ctx::LbWords w = c.lookback_words(nb);
  LIF_LAUNCH(k_union_rows<2>, dim3(nb), dim3(kUR), union_rows_lds(nb, true), c.stream, S, diag_on, nb, nullptr,
             nullptr, rc, cc, ix, stride, id, rowof, w, L);
}

void launch_keep_count_scan(Ctx& c, const int* row_ptr, const double* norms, double tau, int nb, int* out_rp) {
  KeepCount k{row_ptr, norms, tau};
  LIF_LAUNCH(k_count_scan<KeepCount>, dim3(1), dim3(kCS), 0, c.stream, k, nb, out_rp);
}

void launch_filter_count_scan(Ctx& c, const int* row_ptr, const int* col, const int* rlab, const int* clab, int mode,
                              int nb, int* out_rp) {
  FilterCount fc{row_ptr, col, rlab, clab, mode};
  LIF_LAUNCH(k_count_scan<FilterCount>, dim3(1), dim3(kCS), 0, c.stream, fc, nb, out_rp);
}

void launch_intersect_count_scan(Ctx& c, const int* ra, const int* ca, const int* rr, const int* cr, int nb,
                                 int* out_rp) {
  IntersectCount ic{ra, ca, rr, cr};
  LIF_LAUNCH(k_count_scan<IntersectCount>, dim3(1), dim3(kCS), 0, c.stream, ic, nb, out_rp);
}

void launch_compact_gather(Ctx& c, const int* row_ptr, int nb, const int* col, const double* norms, double tau,
                           const int* new_row_ptr, BlkIn blk, int64_t nnzb, int* new_col, BlkOut new_blk) {
  if (nnzb == 0) return;
  LIF_LAUNCH(k_compact_gather, dim3(grid1(nnzb, 256)), dim3(256), 0, c.stream, row_ptr, nb, col, norms, tau,
             new_row_ptr, blk, nnzb, new_col, new_blk);
}

void launch_axpby3_values(Ctx& c, const BlkIn v[3], const double coef[3], const int* ix, int64_t stride,
                          double gamma, const unsigned char* id, const int* row_of, int64_t nnzb, int b, int64_t n,
                          double* store, int* slot, BlkOut out, const int* live, const int* list) {
  if (nnzb == 0) return;
  Val3 V;
  for (int t = 0; t < 3; ++t) {
    V.v[t] = v[t];
    V.coef[t] = coef[t];
  }
  if (list) {
    if (b == 64)
      LIF_LAUNCH((k_axpby_values<64, true>), dim3((unsigned)nnzb), dim3(kWG), 0, c.stream, V, ix, stride, gamma, id,
                 row_of, n, store, slot, out, live, list);
    else
      LIF_LAUNCH((k_axpby_values<32, true>), dim3((unsigned)nnzb), dim3(kWG), 0, c.stream, V, ix, stride, gamma, id,
                 row_of, n, store, slot, out, live, list);
    return;
  }
  if (b == 64)
    LIF_LAUNCH((k_axpby_values<64, false>), dim3((unsigned)nnzb), dim3(kWG), 0, c.stream, V, ix, stride, gamma, id,
               row_of, n, store, slot, out, live, nullptr);
  else
    LIF_LAUNCH((k_axpby_values<32, false>), dim3((unsigned)nnzb), dim3(kWG), 0, c.stream, V, ix, stride, gamma, id,
               row_of, n, store, slot, out, live, nullptr);
}

void launch_block_row_of(Ctx& c, const int* row_ptr, int nb, int64_t nnzb, int* row_of) {
  if (nnzb == 0) return;
  LIF_LAUNCH(k_block_row_of, dim3(nb), dim3(64), 0, c.stream, row_ptr, nb, row_of);
}

void launch_filter_fill(Ctx& c, const int* row_ptr, const int* col, const int* rlab, const int* clab, int mode,
                        const int* new_row_ptr, int nb, int* new_col, int* src) {
  LIF_LAUNCH(k_filter_fill, dim3(grid1(nb, 128)), dim3(128), 0, c.stream, row_ptr, col, rlab, clab, mode,
             new_row_ptr, nb, new_col, src);
}

void launch_transpose_counts(Ctx& c, const int* col, int64_t nnzb, int* counts, const int* live) {
  if (nnzb == 0) return;
  LIF_LAUNCH(k_transpose_counts, dim3(grid1(nnzb, 256)), dim3(256), 0, c.stream, col, nnzb, counts, live);
}

bool transpose_count_scan_fits(int nb) { return (size_t)nb * sizeof(int) <= 48 * 1024; }

void launch_transpose_count_scan(Ctx& c, const int* col, int64_t nnzb, const int* live, int nb, int* tptr,
                                 int* cursor) {
  LIF_LAUNCH(k_transpose_count_scan, dim3(1), dim3(kTC), (size_t)nb * sizeof(int), c.stream, col, nnzb, live, nb, tptr,
             cursor);
}

void launch_transpose_fill(Ctx& c, const int* row_ptr, const int* col, const int* tptr, int nb, int* cursor,
                           int* tcol, int* tsrc) {
  LIF_LAUNCH(k_transpose_fill, dim3(nb), dim3(64), 0, c.stream, row_ptr, col, tptr, nb, cursor, tcol, tsrc);
}

void launch_transpose_sort(Ctx& c, const int* tptr, int nb, const int* icol, const int* isrc, int* ocol,
                           int* osrc) {
  LIF_LAUNCH(k_transpose_sort, dim3(nb), dim3(kWG), 0, c.stream, tptr, icol, isrc, ocol, osrc);
}

void launch_transpose_blocks(Ctx& c, BlkIn blk, const int* src, int64_t nnzb, int b, double* store, BlkOut out,
                             const int* live) {
  if (nnzb == 0) return;
  if (b == 64)
    LIF_LAUNCH(k_transpose_blocks<64>, dim3((unsigned)nnzb), dim3(kWG), 0, c.stream, blk, src, store, out, live);
  else
    LIF_LAUNCH(k_transpose_blocks<32>, dim3((unsigned)nnzb), dim3(kWG), 0, c.stream, blk, src, store, out, live);
}

void launch_segment_sum(Ctx& c, const double* sumsq, const int* row_ptr, const int* rlo, const int* rhi, int nseg,
                        double* out) {
  if (nseg == 0) return;
  LIF_LAUNCH(k_segment_sum, dim3(nseg), dim3(kWG), 0, c.stream, sumsq, row_ptr, rlo, rhi, out);
}

void launch_intersect(Ctx& c, const int* ra, const int* ca, const int* rr, const int* cr, int nb, int* counts,
                      const int* nrp, int* ncol, int* src) {
  LIF_LAUNCH(k_intersect_counts, dim3(grid1(nb, 128)), dim3(128), 0, c.stream, ra, ca, rr, cr, nb, counts, nrp, ncol,
             src);
}

void launch_phi_diag(Ctx& c, const int* row_of, const int* col, int64_t nnzb, int b, double* store, BlkOut blk,
                     const int* live) {
  if (nnzb == 0) return;
  if (b == 64)
    LIF_LAUNCH(k_phi_diag<64>, dim3((unsigned)nnzb), dim3(kWG), 0, c.stream, row_of, col, store, blk, live);
  else
    LIF_LAUNCH(k_phi_diag<32>, dim3((unsigned)nnzb), dim3(kWG), 0, c.stream, row_of, col, store, blk, live);
}

void launch_fill_i32(Ctx& c, int* p, int value, int64_t count) {
  if (count == 0) return;
  LIF_LAUNCH(k_fill_i32, dim3(grid1(count, 256)), dim3(256), 0, c.stream, p, value, count);
}

}  // namespace lif
