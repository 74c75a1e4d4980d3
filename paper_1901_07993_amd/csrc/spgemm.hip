// Block-sparse matrix-matrix product C = op(A) op(B) on b x b dense blocks:
// the sparse multiplication that dominates all three methods of the paper
// (Sec. 2, Sec. 4), with zero blocks skipped as the quad-tree skips null
// children.
//
// Symbolic phase (integer, HBM-bound): one workgroup per block row i of C.
// An operand may carry holes (blocks dropped by its own truncation, left in
// its pattern with null pointers); they take no part in the product.
// The output columns of row i are collected in an LDS bitmap over the nb
// block columns; their number and the number of block products are counted.
// After a host-side prefix sum the fill pass writes C's sorted column list,
// a segment pointer per output block, and the (a, b) block-index pairs of
// each output block in ascending inner index k -- so every output block is
// summed in the same order on every run (no atomics on values).
//
// Numeric phase (FP64 MFMA): one workgroup per output block.  The operand
// blocks of its segment are read through their pointers, contiguous
// fragments straight into registers and the others through one LDS tile
// (see k_numeric_f64); v_mfma_f64_16x16x4f64 accumulates the whole segment
// in registers; the block is written once, with the fused terms of the
// epilogue, together with its Frobenius norm (fixed-order FP64 reduction)
// for the truncation pass.
#include "block_scan.h"
#include "common.h"
#include "lookback.h"
#include "tile_mma.h"

namespace lif {

namespace {

constexpr int kSymWG = 256;

// ---------------------------------------------------------------------------
// symbolic
// ---------------------------------------------------------------------------

// Operands with holes: a block whose pointer is null is absent.  `a`/`b`
// are the block pointers of such an operand (null for one without holes),
// reached through the view's index arrays.
// `jmin`: output columns below it are not formed (the upper block triangle
// of a product: jmin = the row).
struct Holes {
  BlkIn a = nullptr;
  const int* aidx = nullptr;
  BlkIn b = nullptr;
  const int* bidx = nullptr;
  int jmin = 0;
  __device__ bool a_absent(int e) const { return a && !a[aidx ? aidx[e] : e]; }
  __device__ bool b_absent(int f) const { return b && !b[bidx ? bidx[f] : f]; }
};

// `drp`/`dcol` (nullable): a matrix D whose row pattern joins the output
// pattern (the target of a fused term gamma D)
__device__ inline void build_row_bitmap(const int* __restrict__ arp, const int* __restrict__ acol,
                                        const int* __restrict__ brp, const int* __restrict__ bcol, const Holes& h,
                                        const int* __restrict__ drp, const int* __restrict__ dcol, int i,
                                        unsigned* bm, int nwords, int64_t* pcount) {
  for (int w = threadIdx.x; w < nwords; w += kSymWG) bm[w] = 0u;
  __syncthreads();
  if (drp)
    for (int e = drp[i] + threadIdx.x; e < drp[i + 1]; e += kSymWG) {
      const int j = dcol[e];
      if (j < h.jmin) continue;
      atomicOr(&bm[j >> 5], 1u << (j & 31));
    }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool each = h.b || h.jmin > 0;  // products counted one by one
  int64_t p = 0;
  for (int e = arp[i] + wave; e < arp[i + 1]; e += kSymWG / 64) {
    if (h.a_absent(e)) continue;  // uniform over the wave
    const int k = acol[e];
    const int lo = brp[k], hi = brp[k + 1];
    if (!each && lane == 0) p += hi - lo;
    for (int f = lo + lane; f < hi; f += 64) {
      if (h.b_absent(f)) continue;
      const int j = bcol[f];
      if (j < h.jmin) continue;
      if (each) ++p;
      atomicOr(&bm[j >> 5], 1u << (j & 31));
    }
  }
  if (pcount) *pcount = p;
  __syncthreads();
}

__global__ __launch_bounds__(kSymWG) void k_symbolic_count(const int* __restrict__ arp, const int* __restrict__ acol,
                                                           const int* __restrict__ brp, const int* __restrict__ bcol,
                                                           Holes h, const int* __restrict__ drp,
                                                           const int* __restrict__ dcol, int nb, bool upper,
                                                           int* __restrict__ cnt_c, int64_t* __restrict__ cnt_p) {
  extern __shared__ unsigned smem[];
  __shared__ int64_t red_p[kSymWG];
  __shared__ int red_c[kSymWG];
  const int i = blockIdx.x;
  h.jmin = upper ? i : 0;
  const int nwords = (nb + 31) >> 5;
  unsigned* bm = smem;
  int64_t p = 0;
  build_row_bitmap(arp, acol, brp, bcol, h, drp, dcol, i, bm, nwords, &p);
  int c = 0;
  for (int w = threadIdx.x; w < nwords; w += kSymWG) c += __popc(bm[w]);
  red_p[threadIdx.x] = p;
  red_c[threadIdx.x] = c;
  __syncthreads();
  for (int s = kSymWG / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red_p[threadIdx.x] += red_p[threadIdx.x + s];
      red_c[threadIdx.x] += red_c[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    cnt_c[i] = red_c[0];
    cnt_p[i] = red_p[0];
  }
}

// LDS layout of the fill pass: bitmap[nwords] | word_prefix[nwords] | cursor[nb]
// With D, dsrc[e] of each output block is D's block at the same position
// (null where D has none).
__global__ __launch_bounds__(kSymWG) void k_symbolic_fill(const int* __restrict__ arp, const int* __restrict__ acol,
                                                          const int* __restrict__ aidx, const int* __restrict__ brp,
                                                          const int* __restrict__ bcol, const int* __restrict__ bidx,
                                                          BlkIn ablk, BlkIn bblk, bool a_holes, bool b_holes,
                                                          const int* __restrict__ drp,
                                                          const int* __restrict__ dcol, BlkIn dblk, int nb,
                                                          bool upper, const int* __restrict__ crp,
                                                          const int64_t* __restrict__ prp, int* __restrict__ ccol,
                                                          int64_t* __restrict__ seg, BlockPair* __restrict__ pairs,
                                                          BlkOut dsrc, int row0) {
  extern __shared__ unsigned smem[];
  __shared__ int scan_tmp[kSymWG / 64];
  const int i = row0 + (int)blockIdx.x;
  const int row_end = row0 + (int)gridDim.x;  // rows [row0, row_end) in this launch
  const int nwords = (nb + 31) >> 5;
  unsigned* bm = smem;
  int* wp = reinterpret_cast<int*>(smem + nwords);
  int* cur = wp + nwords;
  const Holes h{a_holes ? ablk : nullptr, aidx, b_holes ? bblk : nullptr, bidx, upper ? i : 0};
  build_row_bitmap(arp, acol, brp, bcol, h, drp, dcol, i, bm, nwords, nullptr);

  // exclusive prefix of word popcounts: contiguous chunks per thread
  const int chunk = (nwords + kSymWG - 1) / kSymWG;
  const int w0 = min(nwords, (int)threadIdx.x * chunk), w1 = min(nwords, w0 + chunk);
  int s = 0;
  for (int w = w0; w < w1; ++w) s += __popc(bm[w]);
  int ncols;
  int run = block_exclusive_scan<int, kSymWG>(s, scan_tmp, &ncols);
  for (int w = w0; w < w1; ++w) {
    wp[w] = run;
    run += __popc(bm[w]);
  }
  __syncthreads();

  // output columns in ascending order; zero the per-output product counters
  const int cbase = crp[i];
  for (int w = threadIdx.x; w < nwords; w += kSymWG) {
    unsigned bits = bm[w];
    int r = wp[w];
    while (bits) {
      const int bit = __ffs(bits) - 1;
      const int j = (w << 5) + bit;
      ccol[cbase + r] = j;
      if (dsrc) dsrc[cbase + r] = nullptr;
      cur[r] = 0;
      ++r;
      bits &= bits - 1;
    }
  }
  __syncthreads();

  // D's blocks at their output positions
  if (dsrc)
    for (int e = drp[i] + threadIdx.x; e < drp[i + 1]; e += kSymWG) {
      const int j = dcol[e];
      if (j < h.jmin) continue;
      dsrc[cbase + wp[j >> 5] + __popc(bm[j >> 5] & ((1u << (j & 31)) - 1u))] = dblk[e];
    }

  // products per output block
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int e = arp[i] + wave; e < arp[i + 1]; e += kSymWG / 64) {
    if (h.a_absent(e)) continue;
    const int k = acol[e];
    for (int f = brp[k] + lane; f < brp[k + 1]; f += 64) {
      if (h.b_absent(f)) continue;
      const int j = bcol[f];
      if (j < h.jmin) continue;
      const int r = wp[j >> 5] + __popc(bm[j >> 5] & ((1u << (j & 31)) - 1u));
      atomicAdd(&cur[r], 1);
    }
  }
  __syncthreads();

  // exclusive scan of the per-output counts -> segment starts
  const int c0 = min(ncols, (int)threadIdx.x * ((ncols + kSymWG - 1) / kSymWG));
  const int c1 = min(ncols, c0 + (ncols + kSymWG - 1) / kSymWG);
  int t = 0;
  for (int r = c0; r < c1; ++r) t += cur[r];
  __syncthreads();  // scan_tmp is reused
  int tot;
  int acc = block_exclusive_scan<int, kSymWG>(t, scan_tmp, &tot);
  int64_t prow = prp[i];
  if (i == row_end - 1 && threadIdx.x == 0) seg[crp[row_end]] = prp[row_end];  // closing segment pointer
  for (int r = c0; r < c1; ++r) {
    const int cnt = cur[r];
    seg[cbase + r] = prow + acc;
    cur[r] = acc;
    acc += cnt;
  }
  __syncthreads();

  // pairs in ascending k within each output block: the A row is walked in
  // order; within one k every output column occurs at most once
  // (the same absent blocks as in the counts above)
  for (int e = arp[i]; e < arp[i + 1]; ++e) {
    const int k = acol[e];
    const double* a = ablk[aidx ? aidx[e] : e];
    if (!a_holes || a)  // uniform over the workgroup
      for (int f = brp[k] + threadIdx.x; f < brp[k + 1]; f += kSymWG) {
        const double* bp = bblk[bidx ? bidx[f] : f];
        if (b_holes && !bp) continue;
        const int j = bcol[f];
        if (j < h.jmin) continue;
        const int r = wp[j >> 5] + __popc(bm[j >> 5] & ((1u << (j & 31)) - 1u));
        const int pos = cur[r];
        pairs[prow + pos] = BlockPair{a, bp};
        cur[r] = pos + 1;
      }
    __syncthreads();
  }
}

// The fill pass without a serial walk of the A row.  A pair (e, f) of
// output block r must land after the pairs of r from earlier A entries e'
// (ascending k).  For a run of up to 64 consecutive A entries, every output
// block keeps a 64-bit LDS mask with bit e - e0 set when entry e contributes
// to it; the pair's rank in the block is the popcount of the mask below its
// bit, plus the pairs of earlier runs.  All pairs of a run are placed in
// parallel.  LDS: mask[nb] (64-bit) | bitmap[nwords] | word_prefix[nwords] |
// cursor[nb].
//
// ONEPASS: the counting pass and the scan of the row counts happen in the
// same launch.  The workgroup of row i counts the row's output blocks and
// block products and gets their prefix over the lower rows by a look-back
// over groups of rows (lookback.h); it writes its row pointer itself.  The
// output and pair arrays have the capacities cap_c, cap_p (sized in
// advance): a row that does not fit writes nothing.  The last row writes the
// totals to sizes[0..1] and, when a total exceeds its capacity, raises
// *overflow and leaves the block count crp[nb] at zero; a row whose
// look-back gave up raises *overflow too.  A raised *overflow voids the
// product: the numeric phase then computes nothing and clears the row
// pointers (Epilogue::poison), so that every later reader sees it empty.
// Progress of the look-back relies on workgroups starting in the order of
// their index; were it otherwise, the bounded wait gives up and the
// product is voided, never hung.
struct OnePass {
  Ctx::LbWords lb;  // look-back words: output blocks (a) and block products (b) per row
  int64_t cap_c = 0, cap_p = 0;
  int64_t* sizes = nullptr;
  int* overflow = nullptr;
};

template <bool ONEPASS>
__global__ __launch_bounds__(kSymWG) void k_symbolic_fill_masked(
    const int* __restrict__ arp, const int* __restrict__ acol, const int* __restrict__ aidx,
    const int* __restrict__ brp, const int* __restrict__ bcol, const int* __restrict__ bidx, BlkIn ablk,
    BlkIn bblk, bool a_holes, bool b_holes, const int* __restrict__ drp, const int* __restrict__ dcol, BlkIn dblk,
    int nb, bool upper, int* __restrict__ crp, const int64_t* __restrict__ prp, int* __restrict__ ccol,
    int64_t* __restrict__ seg, BlockPair* __restrict__ pairs, BlkOut dsrc, OnePass op, int row0) {
  extern __shared__ unsigned long long smem64[];
  __shared__ int scan_tmp[kSymWG / 64];
  __shared__ int64_t scan_tmp64[kSymWG / 64];
  __shared__ int64_t off_sh[2];
  __shared__ int flag_sh;
  const int i = row0 + (int)blockIdx.x;  // row0 = 0 in the one-pass form
  const int nwords = (nb + 31) >> 5;
  unsigned long long* mask = smem64;
  unsigned* bm = reinterpret_cast<unsigned*>(smem64 + nb);
  int* wp = reinterpret_cast<int*>(bm + nwords);
  int* cur = wp + nwords;
  const Holes h{a_holes ? ablk : nullptr, aidx, b_holes ? bblk : nullptr, bidx, upper ? i : 0};
  int64_t pcount = 0;
  build_row_bitmap(arp, acol, brp, bcol, h, drp, dcol, i, bm, nwords, ONEPASS ? &pcount : nullptr);

  // exclusive prefix of word popcounts: contiguous chunks per thread
  const int chunk = (nwords + kSymWG - 1) / kSymWG;
  const int w0 = min(nwords, (int)threadIdx.x * chunk), w1 = min(nwords, w0 + chunk);
  int s = 0;
  for (int w = w0; w < w1; ++w) s += __popc(bm[w]);
  int ncols;
  int run = block_exclusive_scan<int, kSymWG>(s, scan_tmp, &ncols);
  for (int w = w0; w < w1; ++w) {
    wp[w] = run;
    run += __popc(bm[w]);
  }

  int64_t prow_count = 0;
  if (ONEPASS) {
    block_exclusive_scan<int64_t, kSymWG>(pcount, scan_tmp64, &prow_count);
    // published now, so that the rows above find it while this row works
    if (threadIdx.x == 0)
      lb_publish(op.lb.ra, op.lb.rb, i, op.lb.epoch, (unsigned long long)ncols, (unsigned long long)prow_count);
  }
  __syncthreads();

  // local work first (needs no offset): clear the per-output counters and
  // masks, count the products of each output block, scan them
  for (int w = threadIdx.x; w < nwords; w += kSymWG) {
    unsigned bits = bm[w];
    int r = wp[w];
    while (bits) {
      cur[r] = 0;
      mask[r] = 0ull;
      ++r;
      bits &= bits - 1;
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int alo = arp[i], ahi = arp[i + 1];
  auto rank = [&](int j) { return wp[j >> 5] + __popc(bm[j >> 5] & ((1u << (j & 31)) - 1u)); };
  // marks the contributions of A entries [e0, e0 + 64) in the masks
  auto mark = [&](int e0) {
    const int e1 = min(ahi, e0 + 64);
    for (int e = e0 + wave; e < e1; e += kSymWG / 64) {
      if (h.a_absent(e)) continue;  // uniform over the wave
      const int k = acol[e];
      const unsigned long long bit = 1ull << (e - e0);
      for (int f = brp[k] + lane; f < brp[k + 1]; f += 64) {
        if (h.b_absent(f)) continue;
        const int j = bcol[f];
        if (j < h.jmin) continue;
        atomicOr(&mask[rank(j)], bit);
      }
    }
  };
  // writes the pairs of A entries [e0, e0 + 64) after cur[r] in each block
  auto place = [&](int e0, int64_t prow) {
    const int e1 = min(ahi, e0 + 64);
    for (int e = e0 + wave; e < e1; e += kSymWG / 64) {
      const double* a = ablk[aidx ? aidx[e] : e];
      if (a_holes && !a) continue;
      const int k = acol[e];
      const unsigned long long below = (1ull << (e - e0)) - 1ull;
      for (int f = brp[k] + lane; f < brp[k + 1]; f += 64) {
        const double* bp = bblk[bidx ? bidx[f] : f];
        if (b_holes && !bp) continue;
        const int j = bcol[f];
        if (j < h.jmin) continue;
        const int r = rank(j);
        pairs[prow + cur[r] + __popcll(mask[r] & below)] = BlockPair{a, bp};
      }
    }
  };
  const bool one_run = ahi - alo <= 64;
  for (int e0 = alo; e0 < ahi; e0 += 64) {
    mark(e0);
    __syncthreads();
    if (!one_run) {
      for (int r = threadIdx.x; r < ncols; r += kSymWG) {
        cur[r] += __popcll(mask[r]);
        mask[r] = 0ull;
      }
      __syncthreads();
    }
  }
  if (one_run)
    for (int r = threadIdx.x; r < ncols; r += kSymWG) cur[r] = __popcll(mask[r]);
  __syncthreads();
  // exclusive scan of the per-output counts: segment starts within the row
  const int c0 = min(ncols, (int)threadIdx.x * ((ncols + kSymWG - 1) / kSymWG));
  const int c1 = min(ncols, c0 + (ncols + kSymWG - 1) / kSymWG);
  {
    int t = 0;
    for (int r = c0; r < c1; ++r) t += cur[r];
    int tot;
    int acc = block_exclusive_scan<int, kSymWG>(t, scan_tmp, &tot);
    for (int r = c0; r < c1; ++r) {
      const int cnt = cur[r];
      cur[r] = acc;
      acc += cnt;
    }
  }

  // the row's offsets in the output and pair arrays
  int cbase;
  int64_t prow;
  bool fits = true;
  if (ONEPASS) {
    if (threadIdx.x < 64) {
      unsigned long long ec = 0, ep = 0;
      const bool ok = lb_resolve2(op.lb.ra, op.lb.rb, op.lb.ga, op.lb.gb, i, nb, op.lb.epoch,
                                  (unsigned long long)ncols, (unsigned long long)prow_count, &ec, &ep);
      if (threadIdx.x == 0) {
        off_sh[0] = (int64_t)ec;
        off_sh[1] = (int64_t)ep;
        flag_sh = ok ? 1 : 0;
        if (!ok) {
          atomicExch(op.overflow, 1);
          atomicExch(op.lb.fail, 1);
        }
      }
    }
    __syncthreads();
    cbase = (int)off_sh[0];
    prow = off_sh[1];
    fits = flag_sh && off_sh[0] + ncols <= op.cap_c && prow + prow_count <= op.cap_p;
    if (threadIdx.x == 0) {
      if (fits) crp[i] = cbase;
      if (i == nb - 1) {
        op.sizes[0] = off_sh[0] + ncols;
        op.sizes[1] = prow + prow_count;
        crp[nb] = fits ? cbase + ncols : 0;
        if (fits) seg[cbase + ncols] = prow + prow_count;  // closing segment pointer
        else atomicExch(op.overflow, 1);
      }
    }
  } else {
    cbase = crp[i];
    prow = prp[i];
    const int row_end = row0 + (int)gridDim.x;  // rows [row0, row_end) in this launch
    if (i == row_end - 1 && threadIdx.x == 0) seg[crp[row_end]] = prp[row_end];  // closing segment pointer
  }
  if (!fits) return;  // uniform over the workgroup

  // output columns in ascending order, segment starts
  for (int w = threadIdx.x; w < nwords; w += kSymWG) {
    unsigned bits = bm[w];
    int r = wp[w];
    while (bits) {
      const int j = (w << 5) + __ffs(bits) - 1;
      ccol[cbase + r] = j;
      if (dsrc) dsrc[cbase + r] = nullptr;
      ++r;
      bits &= bits - 1;
    }
  }
  for (int r = c0; r < c1; ++r) seg[cbase + r] = prow + cur[r];
  __syncthreads();
  if (dsrc)  // D's blocks at their output positions
    for (int e = drp[i] + threadIdx.x; e < drp[i + 1]; e += kSymWG) {
      const int j = dcol[e];
      if (j < h.jmin) continue;
      dsrc[cbase + rank(j)] = dblk[e];
    }

  // pairs: one run reuses its masks; longer rows mark each run again
  if (one_run) {
    place(alo, prow);
    return;
  }
  for (int e0 = alo; e0 < ahi; e0 += 64) {
    mark(e0);
    __syncthreads();
    place(e0, prow);
    __syncthreads();
    for (int r = threadIdx.x; r < ncols; r += kSymWG) {
      cur[r] += __popcll(mask[r]);
      mask[r] = 0ull;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// numeric
// ---------------------------------------------------------------------------

__device__ inline int64_t xcd_remap(int64_t wg, int64_t total) {
  // the dispatcher deals workgroups round-robin to the 8 XCDs; give each XCD
  // a contiguous run of output blocks (they share A blocks of one row and B
  // blocks of neighbouring columns in that XCD's L2)
  const int64_t x = wg & 7, l = wg >> 3;
  const int64_t q = total >> 3, r = total & 7;
  return x * q + (x < r ? x : r) + l;
}

// Output layout of a product tile.  Wave (rb, cb) holds the 32 x 32 quadrant
// as 2 x 2 MFMA tiles (ti, tj).  Where an operand's fragments are contiguous
// in memory (A stored k-major: op(A) = A^T; B stored k-major: op(B) = B), the
// two tiles of that side interleave (rows rb + 2 m + ti, columns
// cb + 2 m + tj), so one 16-byte access carries both tiles' fragments;
// otherwise they are stacked (rb + 16 ti + m, cb + 16 tj + m).  Both numeric
// kernels use this map, so they give bitwise the same blocks and norms.
template <int B, bool TA, bool TB>
struct OutMap {
  static constexpr bool RI = TA, CI = !TB;
  __device__ static int row(const Frag& f, int ti, int m) { return RI ? f.rb + 2 * m + ti : f.rb + 16 * ti + m; }
  __device__ static int col(const Frag& f, int tj, int m) { return CI ? f.cb + 2 * m + tj : f.cb + 16 * tj + m; }
};

// D's elements at the positions this lane holds of C (zeros without D),
// loaded before the products so that they arrive during them.
template <int B, bool TA, bool TB>
__device__ __attribute__((always_inline)) inline void load_d(const Frag& f, const double* __restrict__ Db,
                                                             double (&d)[2][2][4]) {
  using M = OutMap<B, TA, TB>;
  if (Db) {  // uniform across the workgroup
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const auto* q = gptr(Db + M::row(f, ti, 4 * r + f.kq) * B);
        if (M::CI) {
          const v2d dv = *gptr(reinterpret_cast<const v2d*>(Db + M::row(f, ti, 4 * r + f.kq) * B + M::col(f, 0, f.l16)));
          d[ti][0][r] = dv.x;
          d[ti][1][r] = dv.y;
        } else {
          d[ti][0][r] = q[M::col(f, 0, f.l16)];
          d[ti][1][r] = q[M::col(f, 1, f.l16)];
        }
      }
  } else {
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r) d[ti][tj][r] = 0.0;
  }
}

// The block alpha A B (+ gamma D when HAS_D, D's elements in d), its FP64
// sum of squares in a fixed order, its norm and its pointer; the values are
// written once the norm has decided whether (and where) the block is kept.
template <int B, bool TA, bool TB, bool HAS_D>
__device__ __attribute__((always_inline)) inline void numeric_epilogue(const v4d (&acc)[2][2], const Frag& f,
                                                                       int64_t blk, double* __restrict__ C,
                                                                       BlkOut Cp, double* __restrict__ norms,
                                                                       const Epilogue& epi,
                                                                       const double (&d)[2][2][4], double* red) {
  using Cfg = TileCfg<B>;
  using M = OutMap<B, TA, TB>;
  double v[2][2][4];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        v[ti][tj][r] = epi.alpha * acc[ti][tj][r];
        if (HAS_D) v[ti][tj][r] += epi.gamma * d[ti][tj][r];
      }
  double ss = 0.0;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) ss += v[ti][tj][r] * v[ti][tj][r];
  for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
  if (f.lane == 0) red[f.wave] = ss;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < Cfg::WAVES; ++w) t += red[w];
    const double nrm = sqrt(t);
    if (norms) norms[blk] = nrm;
    const int64_t s = output_slot(epi, blk, nrm);
    Cp[blk] = s >= 0 ? C + s * B * B : nullptr;
    red[Cfg::WAVES] = __longlong_as_double(s);
  }
  __syncthreads();
  const int64_t slot = __double_as_longlong(red[Cfg::WAVES]);
  if (slot < 0) return;  // dropped: never written
  double* Cb = C + slot * B * B;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = M::row(f, ti, 4 * r + f.kq);
      if (M::CI) {
        *reinterpret_cast<v2d*>(Cb + row * B + M::col(f, 0, f.l16)) = v2d{v[ti][0][r], v[ti][1][r]};
      } else {
        Cb[row * B + M::col(f, 0, f.l16)] = v[ti][0][r];
        Cb[row * B + M::col(f, 1, f.l16)] = v[ti][1][r];
      }
    }
}

// Numeric kernel, one workgroup per output block.  Fragments whose elements
// are contiguous in memory are loaded straight from global memory into
// registers (16 bytes per lane: both tiles of a side); only an operand read
// across its rows (op(A) = A, op(B) = B^T) is staged in LDS, as stored.
// With at most one LDS tile, two or three workgroups share a CU and hide
// each other's load latency -- on the sparse products of the refinement
// (one to three block products per output block) and on dense ones (219
// per block) alike this beat a double-buffered two-tile LDS pipeline.
template <int B, bool TA, bool TB, bool HAS_D>
__global__ __launch_bounds__(TileCfg<B>::THREADS) void k_numeric_f64(const int64_t* __restrict__ seg,
                                                                        const BlockPair* __restrict__ pairs,
                                                                        const int* __restrict__ live,
                                                                        double* __restrict__ C, BlkOut Cp,
                                                                        double* __restrict__ norms, Epilogue epi) {
  using Cfg = TileCfg<B>;
  constexpr bool A_LDS = !TA, B_LDS = TB;
  constexpr int KS = B / 4;
  __shared__ __attribute__((aligned(16))) double As[A_LDS ? Cfg::LDS_DOUBLES : 2];
  __shared__ __attribute__((aligned(16))) double Bs[B_LDS ? Cfg::LDS_DOUBLES : 2];
  __shared__ double red[Cfg::WAVES + 1];  // partial sums, then the output slot
  const int64_t nlive = live_blocks(live, epi);
  if ((int64_t)blockIdx.x >= nlive) return;
  const int64_t blk = xcd_remap(blockIdx.x, nlive);
  const int64_t p0 = seg[blk], p1 = seg[blk + 1];
  const Frag f = frag_coords<B>();
  double d[2][2][4];
  if (HAS_D) load_d<B, TA, TB>(f, epi.dsrc[blk], d);
  v4d acc[2][2];
  acc_zero(acc);
  for (int64_t p = p0; p < p1; ++p) {
    const BlockPair pr = pairs[p];
    v2d ra[Cfg::V2], rbv[Cfg::V2];
    v2d ad[KS], bd[KS];
    if (A_LDS) {
      tile_load<B>(pr.a, ra);
    } else {
#pragma unroll
      for (int kk = 0; kk < KS; ++kk)
        ad[kk] = *gptr(reinterpret_cast<const v2d*>(pr.a + (4 * kk + f.kq) * B + f.rb + 2 * f.l16));
    }
    if (B_LDS) {
      tile_load<B>(pr.b, rbv);
    } else {
#pragma unroll
      for (int kk = 0; kk < KS; ++kk)
        bd[kk] = *gptr(reinterpret_cast<const v2d*>(pr.b + (4 * kk + f.kq) * B + f.cb + 2 * f.l16));
    }
    if (A_LDS || B_LDS) {
      if (p > p0) __syncthreads();  // the previous pair's fragment reads are done
      if (A_LDS) tile_store<B>(As, ra, true);
      if (B_LDS) tile_store<B>(Bs, rbv, true);
      __syncthreads();
    }
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      const int k = 4 * kk + f.kq;
      constexpr int LD = Cfg::LD;
      const double a0 = A_LDS ? As[(f.rb + f.l16) * LD + k] : ad[kk].x;
      const double a1 = A_LDS ? As[(f.rb + 16 + f.l16) * LD + k] : ad[kk].y;
      const double b0 = B_LDS ? Bs[(f.cb + f.l16) * LD + k] : bd[kk].x;
      const double b1 = B_LDS ? Bs[(f.cb + 16 + f.l16) * LD + k] : bd[kk].y;
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
  }
  numeric_epilogue<B, TA, TB, HAS_D>(acc, f, blk, C, Cp, norms, epi, d, red);
}

// The same with operand sharing for large products: a workgroup computes G
// consecutive output blocks, walking their lists of block products together
// -- at each step the smallest A block pointer among the lists' next products
// is loaded (and staged) once and the products of every list whose next
// product has that A block run against it.  Each list is consumed in its own
// order with the MFMA sequence of k_numeric_f64, so every block is bitwise
// the same; A blocks stored in block order (as sums, products and compaction
// leave them) are shared between the outputs of a row.
template <int B, bool TA, bool TB, bool HAS_D, int G>
__global__ __launch_bounds__(TileCfg<B>::THREADS) void k_numeric_f64_group(const int64_t* __restrict__ seg,
                                                                              const BlockPair* __restrict__ pairs,
                                                                              const int* __restrict__ live,
                                                                              double* __restrict__ C, BlkOut Cp,
                                                                              double* __restrict__ norms,
                                                                              Epilogue epi, int64_t nblocks) {
  using Cfg = TileCfg<B>;
  constexpr bool A_LDS = !TA, B_LDS = TB;
  constexpr int KS = B / 4;
  __shared__ __attribute__((aligned(16))) double As[A_LDS ? Cfg::LDS_DOUBLES : 2];
  __shared__ __attribute__((aligned(16))) double Bs[B_LDS ? Cfg::LDS_DOUBLES : 2];
  __shared__ double red[Cfg::WAVES + 1];
  // the output blocks of the launch: *live, else all nblocks (the grid has
  // one workgroup per G of them); none for a voided product, whose row
  // pointers workgroup 0 clears
  int64_t nlive;
  if (epi.poison && *epi.poison) {
    if (blockIdx.x == 0)
      for (int r = threadIdx.x; r <= epi.nrows; r += blockDim.x) epi.rows[r] = 0;
    nlive = 0;
  } else {
    nlive = live ? min((int64_t)*live, nblocks) : nblocks;
  }
  const int64_t ngroups = (nlive + G - 1) / G;
  if ((int64_t)blockIdx.x >= ngroups) return;
  const int64_t e0 = xcd_remap(blockIdx.x, ngroups) * G;
  const Frag f = frag_coords<B>();
  v4d acc[G][2][2];
  int64_t pp[G], pe[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const bool in = e0 + g < nlive;
    pp[g] = in ? seg[e0 + g] : 0;
    pe[g] = in ? seg[e0 + g + 1] : 0;
    acc_zero(acc[g]);
  }
  bool staged = false;  // LDS holds tiles that MFMAs of the workgroup may still read
  for (;;) {
    uintptr_t amin = ~uintptr_t(0);
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (pp[g] < pe[g]) amin = min(amin, reinterpret_cast<uintptr_t>(pairs[pp[g]].a));
    if (amin == ~uintptr_t(0)) break;
    const double* pa = reinterpret_cast<const double*>(amin);
    v2d ad[KS];
    if (A_LDS) {
      v2d ra[Cfg::V2];
      tile_load<B>(pa, ra);
      if (staged) __syncthreads();
      tile_store<B>(As, ra, true);
      __syncthreads();
      staged = true;
    } else {
#pragma unroll
      for (int kk = 0; kk < KS; ++kk)
        ad[kk] = *gptr(reinterpret_cast<const v2d*>(pa + (4 * kk + f.kq) * B + f.rb + 2 * f.l16));
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      // uniform over the workgroup: the lists and their heads are shared
      if (!(pp[g] < pe[g] && reinterpret_cast<uintptr_t>(pairs[pp[g]].a) == amin)) continue;
      const double* pb = pairs[pp[g]].b;
      v2d bd[KS];
      if (B_LDS) {
        v2d rbv[Cfg::V2];
        tile_load<B>(pb, rbv);
        if (staged) __syncthreads();
        tile_store<B>(Bs, rbv, true);
        __syncthreads();
        staged = true;
      } else {
#pragma unroll
        for (int kk = 0; kk < KS; ++kk)
          bd[kk] = *gptr(reinterpret_cast<const v2d*>(pb + (4 * kk + f.kq) * B + f.cb + 2 * f.l16));
      }
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) {
        const int k = 4 * kk + f.kq;
        constexpr int LD = Cfg::LD;
        const double a0 = A_LDS ? As[(f.rb + f.l16) * LD + k] : ad[kk].x;
        const double a1 = A_LDS ? As[(f.rb + 16 + f.l16) * LD + k] : ad[kk].y;
        const double b0 = B_LDS ? Bs[(f.cb + f.l16) * LD + k] : bd[kk].x;
        const double b1 = B_LDS ? Bs[(f.cb + 16 + f.l16) * LD + k] : bd[kk].y;
        acc[g][0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[g][0][0], 0, 0, 0);
        acc[g][0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[g][0][1], 0, 0, 0);
        acc[g][1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[g][1][0], 0, 0, 0);
        acc[g][1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[g][1][1], 0, 0, 0);
      }
      ++pp[g];
    }
  }
#pragma unroll
  for (int g = 0; g < G; ++g)
    if (e0 + g < nlive) {
      double d[2][2][4];
      if (HAS_D) load_d<B, TA, TB>(f, epi.dsrc[e0 + g], d);
      numeric_epilogue<B, TA, TB, HAS_D>(acc[g], f, e0 + g, C, Cp, norms, epi, d, red);
    }
}

// outputs per workgroup of the FP64 product on large products (1: one
// each).  Two: 4 % less time on the FP64 factorizations of the water
// clusters; four leaves one workgroup per SIMD and is 17 % slower.
#ifndef LIF_F64_GROUP
#define LIF_F64_GROUP 2
#endif
constexpr int kF64Group = LIF_F64_GROUP;
// products with at least this many output blocks use the grouped kernel
constexpr int64_t kF64GroupMin = 16384;

template <int B, bool TA, bool TB>
void launch_numeric_t(Ctx& c, dim3 grid, const int64_t* seg, const BlockPair* pairs, const int* live, double* C,
                      BlkOut Cp, double* norms, const Epilogue& epi) {
  const dim3 block(TileCfg<B>::THREADS);
  const int64_t nnzc = grid.x;
  // op(A) = A^T keeps one output block per workgroup: its A fragments come
  // straight from memory, and with two outputs' accumulators beside them
  // the grouped form leaves one workgroup per SIMD (measured: 4.6 % more
  // time for the BF16 schedule on water-10 000, where these products are
  // most of the FP64 work; FP64 alone unchanged)
  if (kF64Group > 1 && nnzc >= kF64GroupMin && !TA) {
    const dim3 ggrid((unsigned)((nnzc + kF64Group - 1) / kF64Group));
    if (epi.dsrc)
      hipLaunchKernelGGL((k_numeric_f64_group<B, TA, TB, true, kF64Group>), ggrid, block, 0, c.stream, seg, pairs,
                         live, C, Cp, norms, epi, nnzc);
    else
      hipLaunchKernelGGL((k_numeric_f64_group<B, TA, TB, false, kF64Group>), ggrid, block, 0, c.stream, seg, pairs,
                         live, C, Cp, norms, epi, nnzc);
    return;
  }
  if (epi.dsrc)
    hipLaunchKernelGGL((k_numeric_f64<B, TA, TB, true>), grid, block, 0, c.stream, seg, pairs, live, C, Cp, norms,
                       epi);
  else
    hipLaunchKernelGGL((k_numeric_f64<B, TA, TB, false>), grid, block, 0, c.stream, seg, pairs, live, C, Cp, norms,
                       epi);
}

template <int B>
void launch_numeric_b(Ctx& c, bool ta, bool tb, const int64_t* seg, const BlockPair* pairs, int64_t nnzc,
                      const int* live, double* C, BlkOut Cp, double* norms, const Epilogue& epi) {
  const dim3 grid((unsigned)nnzc);
  if (!ta && !tb)
    launch_numeric_t<B, false, false>(c, grid, seg, pairs, live, C, Cp, norms, epi);
  else if (ta && !tb)
    launch_numeric_t<B, true, false>(c, grid, seg, pairs, live, C, Cp, norms, epi);
  else if (!ta && tb)
    launch_numeric_t<B, false, true>(c, grid, seg, pairs, live, C, Cp, norms, epi);
  else
    launch_numeric_t<B, true, true>(c, grid, seg, pairs, live, C, Cp, norms, epi);
  LIF_HIP(hipGetLastError());
}

}  // namespace

size_t symbolic_lds_bytes(int nb, bool fill) {
  const size_t nwords = (size_t)(nb + 31) / 32;
  return fill ? nwords * 8 + (size_t)nb * 4 : nwords * 4;
}

// the masked fill while its LDS (masks added) stays within 64 KiB, i.e. up
// to about 5000 block rows; the serial-walk fill above that
static size_t masked_fill_lds_bytes(int nb) { return symbolic_lds_bytes(nb, true) + (size_t)nb * 8; }
constexpr size_t kMaskedFillLds = 64 * 1024;

static void allow_lds(const void* fn, size_t bytes) {
  if (bytes > 48 * 1024)
    LIF_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

void launch_symbolic_count(Ctx& c, const int* arp, const int* acol, const int* aidx, const int* brp,
                           const int* bcol, const int* bidx, BlkIn ahole, BlkIn bhole, const int* drp,
                           const int* dcol, int nb, int* cnt_c, int64_t* cnt_p, bool upper) {
  allow_lds((const void*)k_symbolic_count, symbolic_lds_bytes(nb, false));
  const Holes h{ahole, aidx, bhole, bidx};
  hipEvent_t t0 = c.timed_begin(2);
  hipLaunchKernelGGL(k_symbolic_count, dim3(nb), dim3(kSymWG), symbolic_lds_bytes(nb, false), c.stream, arp, acol,
                     brp, bcol, h, drp, dcol, nb, upper, cnt_c, cnt_p);
  LIF_HIP(hipGetLastError());
  c.timed_end(t0, Ctx::Symbolic);
}

void launch_symbolic_fill(Ctx& c, const int* arp, const int* acol, const int* aidx, const int* brp, const int* bcol,
                          const int* bidx, BlkIn ablk, BlkIn bblk, bool a_holes, bool b_holes, const int* drp,
                          const int* dcol, BlkIn dblk, int nb, const int* crp, const int64_t* prp, int* ccol,
                          int64_t* seg, BlockPair* pairs, BlkOut dsrc, bool upper, int row0, int rows) {
  if (rows < 0) rows = nb - row0;
  LIF_REQUIRE(row0 >= 0 && rows >= 1 && row0 + rows <= nb, LIF_ERR_INVALID, "symbolic fill: row range");
  hipEvent_t t0 = c.timed_begin(2);
  if (masked_fill_lds_bytes(nb) <= kMaskedFillLds) {
    allow_lds((const void*)k_symbolic_fill_masked<false>, masked_fill_lds_bytes(nb));
    hipLaunchKernelGGL(k_symbolic_fill_masked<false>, dim3(rows), dim3(kSymWG), masked_fill_lds_bytes(nb), c.stream,
                       arp, acol, aidx, brp, bcol, bidx, ablk, bblk, a_holes, b_holes, drp, dcol, dblk, nb, upper,
                       const_cast<int*>(crp), prp, ccol, seg, pairs, dsrc, OnePass{}, row0);
    LIF_HIP(hipGetLastError());
    c.timed_end(t0, Ctx::Symbolic);
    return;
  }
  allow_lds((const void*)k_symbolic_fill, symbolic_lds_bytes(nb, true));
  hipLaunchKernelGGL(k_symbolic_fill, dim3(rows), dim3(kSymWG), symbolic_lds_bytes(nb, true), c.stream, arp, acol,
                     aidx, brp, bcol, bidx, ablk, bblk, a_holes, b_holes, drp, dcol, dblk, nb, upper, crp, prp, ccol,
                     seg, pairs, dsrc, row0);
  LIF_HIP(hipGetLastError());
  c.timed_end(t0, Ctx::Symbolic);
}

bool symbolic_onepass_fits(int nb) { return masked_fill_lds_bytes(nb) <= kMaskedFillLds; }

void launch_symbolic_onepass(Ctx& c, const int* arp, const int* acol, const int* aidx, const int* brp,
                             const int* bcol, const int* bidx, BlkIn ablk, BlkIn bblk, bool a_holes, bool b_holes,
                             const int* drp, const int* dcol, BlkIn dblk, int nb, int64_t cap_c, int64_t cap_p,
                             int* crp, int* ccol, int64_t* seg, BlockPair* pairs, BlkOut dsrc, int64_t* sizes,
                             int* overflow, bool upper) {
  OnePass op;
  op.lb = c.lookback_words(nb);
  op.cap_c = cap_c;
  op.cap_p = cap_p;
  op.sizes = sizes;
  op.overflow = overflow;
  allow_lds((const void*)k_symbolic_fill_masked<true>, masked_fill_lds_bytes(nb));
  hipEvent_t t0 = c.timed_begin(2);
  hipLaunchKernelGGL(k_symbolic_fill_masked<true>, dim3(nb), dim3(kSymWG), masked_fill_lds_bytes(nb), c.stream, arp,
                     acol, aidx, brp, bcol, bidx, ablk, bblk, a_holes, b_holes, drp, dcol, dblk, nb, upper, crp,
                     nullptr, ccol, seg, pairs, dsrc, op, 0);
  LIF_HIP(hipGetLastError());
  c.timed_end(t0, Ctx::Symbolic);
}

void launch_numeric(Ctx& c, int prec, bool ta, bool tb, const int64_t* seg, const BlockPair* pairs,
                    int64_t nnzc, const int* live, int b, double* C, BlkOut Cp, double* norms, const Epilogue& epi) {
  nnzc = std::max<int64_t>(nnzc, epi.poison ? 1 : 0);  // a voided product still clears its row pointers
  if (nnzc == 0) return;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c.timing) {
    e0 = c.take_event();
    e1 = c.take_event();
    LIF_HIP(hipEventRecord(e0, c.stream));
  }
  if (prec != LIF_FP64)
    launch_numeric_mixed(c, prec, seg, pairs, nnzc, live, b, C, Cp, norms, epi);
  else if (b == 64)
    launch_numeric_b<64>(c, ta, tb, seg, pairs, nnzc, live, C, Cp, norms, epi);
  else
    launch_numeric_b<32>(c, ta, tb, seg, pairs, nnzc, live, C, Cp, norms, epi);
  if (c.timing) {
    LIF_HIP(hipEventRecord(e1, c.stream));
    c.ev_pending.emplace_back(e0, e1);
    c.ev_lowp.push_back((char)prec);
    c.ev_cat.push_back(Ctx::Gemm);
  }
  c.stats.gemm_launches += 1;
  if (prec != LIF_FP64) c.stats.gemm_launches_lowp += 1;
  if (prec == LIF_MIXED_FP32) c.stats.gemm_launches_f32 += 1;
}

}  // namespace lif
