// Block-sparse matrix-matrix product C = op(A) op(B) on b x b dense blocks:
// the sparse multiplication that dominates all three methods of the paper
// (Sec. 2, Sec. 4), with zero blocks skipped as the quad-tree skips null
// children.
//
// Symbolic phase (integer, HBM-bound): one workgroup per block row i of C.
// The output columns of row i are collected in an LDS bitmap over the nb
// block columns; their number and the number of block products are counted.
// After a host-side prefix sum the fill pass writes C's sorted column list,
// a segment pointer per output block, and the (a, b) block-index pairs of
// each output block in ascending inner index k -- so every output block is
// summed in the same order on every run (no atomics on values).
//
// Numeric phase (FP64 MFMA): one workgroup per output block.  The operand
// blocks of its segment stream through two LDS stages (see k_numeric_f64);
// v_mfma_f64_16x16x4f64 accumulates the whole segment in registers; the
// block is written once, together with its Frobenius norm (fixed-order FP64
// reduction) for the truncation pass.
#include "common.h"
#include "tile_mma.h"

namespace lif {

namespace {

constexpr int kSymWG = 256;

// ---------------------------------------------------------------------------
// symbolic
// ---------------------------------------------------------------------------

// `diag_on` (nullable): rows whose diagonal block joins the pattern whether
// or not a product reaches it (the target of a fused identity term)
__device__ inline void build_row_bitmap(const int* __restrict__ arp, const int* __restrict__ acol,
                                        const int* __restrict__ brp, const int* __restrict__ bcol,
                                        const unsigned char* __restrict__ diag_on, int i, unsigned* bm, int nwords,
                                        int64_t* pcount) {
  for (int w = threadIdx.x; w < nwords; w += kSymWG) bm[w] = 0u;
  __syncthreads();
  if (threadIdx.x == 0 && diag_on && diag_on[i]) atomicOr(&bm[i >> 5], 1u << (i & 31));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t p = 0;
  for (int e = arp[i] + wave; e < arp[i + 1]; e += kSymWG / 64) {
    const int k = acol[e];
    const int lo = brp[k], hi = brp[k + 1];
    if (lane == 0) p += hi - lo;
    for (int f = lo + lane; f < hi; f += 64) {
      const int j = bcol[f];
      atomicOr(&bm[j >> 5], 1u << (j & 31));
    }
  }
  if (pcount) *pcount = p;
  __syncthreads();
}

__global__ __launch_bounds__(kSymWG) void k_symbolic_count(const int* __restrict__ arp, const int* __restrict__ acol,
                                                           const int* __restrict__ brp, const int* __restrict__ bcol,
                                                           const unsigned char* __restrict__ diag_on, int nb,
                                                           int* __restrict__ cnt_c, int64_t* __restrict__ cnt_p) {
  extern __shared__ unsigned smem[];
  __shared__ int64_t red_p[kSymWG];
  __shared__ int red_c[kSymWG];
  const int i = blockIdx.x;
  const int nwords = (nb + 31) >> 5;
  unsigned* bm = smem;
  int64_t p = 0;
  build_row_bitmap(arp, acol, brp, bcol, diag_on, i, bm, nwords, &p);
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
// With `diag_on`, dflag[e] of each output block is the number of real rows
// of a diagonal block that takes the identity term (0 for the others).
__global__ __launch_bounds__(kSymWG) void k_symbolic_fill(const int* __restrict__ arp, const int* __restrict__ acol,
                                                          const int* __restrict__ aidx, const int* __restrict__ brp,
                                                          const int* __restrict__ bcol, const int* __restrict__ bidx,
                                                          BlkIn ablk, BlkIn bblk,
                                                          const unsigned char* __restrict__ diag_on, int b,
                                                          int64_t n, int nb, const int* __restrict__ crp,
                                                          const int64_t* __restrict__ prp, int* __restrict__ ccol,
                                                          int64_t* __restrict__ seg, BlockPair* __restrict__ pairs,
                                                          unsigned char* __restrict__ dflag) {
  extern __shared__ unsigned smem[];
  __shared__ int scan_tmp[kSymWG];
  const int i = blockIdx.x;
  const int nwords = (nb + 31) >> 5;
  unsigned* bm = smem;
  int* wp = reinterpret_cast<int*>(smem + nwords);
  int* cur = wp + nwords;
  build_row_bitmap(arp, acol, brp, bcol, diag_on, i, bm, nwords, nullptr);
  const int drows = (diag_on && diag_on[i]) ? (int)min<int64_t>(b, n - (int64_t)i * b) : 0;

  // exclusive prefix of word popcounts: contiguous chunks per thread
  const int chunk = (nwords + kSymWG - 1) / kSymWG;
  const int w0 = min(nwords, (int)threadIdx.x * chunk), w1 = min(nwords, w0 + chunk);
  int s = 0;
  for (int w = w0; w < w1; ++w) s += __popc(bm[w]);
  scan_tmp[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < kSymWG; off <<= 1) {
    int v = (threadIdx.x >= off) ? scan_tmp[threadIdx.x - off] : 0;
    __syncthreads();
    scan_tmp[threadIdx.x] += v;
    __syncthreads();
  }
  const int ncols = scan_tmp[kSymWG - 1];
  int run = threadIdx.x ? scan_tmp[threadIdx.x - 1] : 0;
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
      if (dflag) dflag[cbase + r] = (unsigned char)(j == i ? drows : 0);
      cur[r] = 0;
      ++r;
      bits &= bits - 1;
    }
  }
  __syncthreads();

  // products per output block
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int e = arp[i] + wave; e < arp[i + 1]; e += kSymWG / 64) {
    const int k = acol[e];
    for (int f = brp[k] + lane; f < brp[k + 1]; f += 64) {
      const int j = bcol[f];
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
  __syncthreads();
  scan_tmp[threadIdx.x] = t;
  __syncthreads();
  for (int off = 1; off < kSymWG; off <<= 1) {
    int v = (threadIdx.x >= off) ? scan_tmp[threadIdx.x - off] : 0;
    __syncthreads();
    scan_tmp[threadIdx.x] += v;
    __syncthreads();
  }
  int64_t prow = prp[i];
  if (i == nb - 1 && threadIdx.x == 0) seg[crp[nb]] = prp[nb];  // closing segment pointer
  int acc = threadIdx.x ? scan_tmp[threadIdx.x - 1] : 0;
  for (int r = c0; r < c1; ++r) {
    const int cnt = cur[r];
    seg[cbase + r] = prow + acc;
    cur[r] = acc;
    acc += cnt;
  }
  __syncthreads();

  // pairs in ascending k within each output block: the A row is walked in
  // order; within one k every output column occurs at most once
  for (int e = arp[i]; e < arp[i + 1]; ++e) {
    const int k = acol[e];
    const double* a = ablk[aidx ? aidx[e] : e];
    for (int f = brp[k] + threadIdx.x; f < brp[k + 1]; f += kSymWG) {
      const int j = bcol[f];
      const int r = wp[j >> 5] + __popc(bm[j >> 5] & ((1u << (j & 31)) - 1u));
      const int pos = cur[r];
      pairs[prow + pos] = BlockPair{a, bblk[bidx ? bidx[f] : f]};
      cur[r] = pos + 1;
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

// Operand blocks are stored into LDS as they are (row-major, 16-byte
// stores); op() is applied when the MFMA fragments are read: a fragment is
// either 16 consecutive doubles or 16 doubles one LDS row (66 doubles) apart,
// both conflict-free within a quarter-wave.  Two LDS stages: while the
// waves multiply the tiles of pair p, the tiles of pair p+1 are written to
// the other stage and those of pair p+2 are loaded into registers, with one
// barrier per pair.
template <int B, bool TA, bool TB>
__device__ inline void mma_stage(const double* __restrict__ As, const double* __restrict__ Bs, const Frag& f,
                                 v4d (&acc)[2][2]) {
  constexpr int LD = TileCfg<B>::LD;
#pragma unroll 4
  for (int kk = 0; kk < B / 4; ++kk) {
    const int k = 4 * kk + f.kq;
    // op(A)[i][k]: A[i][k] (row i of the stored block) or A[k][i] (row k)
    const double a0 = TA ? As[k * LD + f.rb + f.l16] : As[(f.rb + f.l16) * LD + k];
    const double a1 = TA ? As[k * LD + f.rb + 16 + f.l16] : As[(f.rb + 16 + f.l16) * LD + k];
    // op(B)[k][j]: B[k][j] or B[j][k]
    const double b0 = TB ? Bs[(f.cb + f.l16) * LD + k] : Bs[k * LD + f.cb + f.l16];
    const double b1 = TB ? Bs[(f.cb + 16 + f.l16) * LD + k] : Bs[k * LD + f.cb + 16 + f.l16];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
}

// STAGES = 2 for long segments (the pipeline above); STAGES = 1 halves the
// LDS so that two workgroups share a CU, for products whose output blocks
// sum only one or two block products (their latency is hidden across
// workgroups instead): store, barrier, prefetch the next pair, multiply.
template <int B, bool TA, bool TB, int STAGES>
__global__ __launch_bounds__(TileCfg<B>::THREADS) void k_numeric_f64(const int64_t* __restrict__ seg,
                                                                     const BlockPair* __restrict__ pairs,
                                                                     const int* __restrict__ live,
                                                                     double* __restrict__ C, BlkOut Cp,
                                                                     double* __restrict__ norms, Epilogue epi) {
  using Cfg = TileCfg<B>;
  __shared__ double As[STAGES][Cfg::LDS_DOUBLES];
  __shared__ double Bs[STAGES][Cfg::LDS_DOUBLES];
  __shared__ double red[Cfg::WAVES];
  // the grid may exceed the live output count (capacity fixed before the
  // count was known); the XCD remap runs over the live blocks only
  const int64_t nlive = *live;
  if ((int64_t)blockIdx.x >= nlive) return;
  const int64_t blk = xcd_remap(blockIdx.x, nlive);
  const int64_t p0 = seg[blk], p1 = seg[blk + 1];
  const Frag f = frag_coords<B>();

  v4d acc[2][2];
  acc_zero(acc);
  // The loop body has no branches around the prefetch registers (the
  // prefetch index is clamped to the last pair; the surplus loads and the
  // last surplus LDS store are never read), which keeps them in VGPRs.
  v2d ra[Cfg::V2], rbv[Cfg::V2];
  const int64_t plast = p1 - 1;
  if (p1 > p0 && STAGES == 1) {
    {
      const BlockPair pr = pairs[p0];
      tile_load<B>(pr.a, ra);
      tile_load<B>(pr.b, rbv);
    }
    for (int64_t p = p0; p < p1; ++p) {
      if (p > p0) __syncthreads();  // the previous pair's fragment reads are done
      tile_store<B>(As[0], ra, true);
      tile_store<B>(Bs[0], rbv, true);
      __syncthreads();
      const BlockPair pr = pairs[min(p + 1, plast)];
      tile_load<B>(pr.a, ra);
      tile_load<B>(pr.b, rbv);
      mma_stage<B, TA, TB>(As[0], Bs[0], f, acc);
    }
  } else if (p1 > p0) {  // a diagonal block of a fused identity term may have no products
    {
      const BlockPair pr = pairs[p0];
      tile_load<B>(pr.a, ra);
      tile_load<B>(pr.b, rbv);
    }
    tile_store<B>(As[0], ra, true);
    tile_store<B>(Bs[0], rbv, true);
    {
      const BlockPair pr = pairs[min(p0 + 1, plast)];
      tile_load<B>(pr.a, ra);
      tile_load<B>(pr.b, rbv);
    }
    int stage = 0;
    for (int64_t p = p0; p < p1; ++p) {
      __syncthreads();  // stage p visible; stage p+1's previous readers done
      tile_store<B>(As[(stage ^ 1) % STAGES], ra, true);
      tile_store<B>(Bs[(stage ^ 1) % STAGES], rbv, true);
      const BlockPair pr = pairs[min(p + 2, plast)];
      tile_load<B>(pr.a, ra);
      tile_load<B>(pr.b, rbv);
      mma_stage<B, TA, TB>(As[stage % STAGES], Bs[stage % STAGES], f, acc);
      stage ^= 1;
    }
  }

  // epilogue: FP64 sum of squares in a fixed order, then the block
  double ss = 0.0;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) ss += acc[ti][tj][r] * acc[ti][tj][r];
  for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
  if (f.lane == 0) red[f.wave] = ss;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < Cfg::WAVES; ++w) t += red[w];
  const double nrm = sqrt(t);
  const int dr = epi.dflag ? epi.dflag[blk] : 0;
  const bool keep = dr == 0 || !(epi.tau > 0.0) || nrm >= epi.tau;
  double* Cb = C + blk * B * B;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = acc_row(f, ti, r), col = acc_col(f, tj);
        double v = keep ? acc[ti][tj][r] : 0.0;
        if (row == col && row < dr) v += epi.gamma;
        Cb[row * B + col] = v;
      }
  if (threadIdx.x == 0) {
    norms[blk] = dr ? INFINITY : nrm;
    Cp[blk] = Cb;
  }
}

template <int B, int STAGES>
void launch_numeric_s(Ctx& c, bool ta, bool tb, const int64_t* seg, const BlockPair* pairs, int64_t nnzc,
                      const int* live, double* C, BlkOut Cp, double* norms, const Epilogue& epi) {
  using Cfg = TileCfg<B>;
  dim3 grid((unsigned)nnzc), block(Cfg::THREADS);
  if (!ta && !tb)
    hipLaunchKernelGGL((k_numeric_f64<B, false, false, STAGES>), grid, block, 0, c.stream, seg, pairs, live, C, Cp,
                       norms, epi);
  else if (ta && !tb)
    hipLaunchKernelGGL((k_numeric_f64<B, true, false, STAGES>), grid, block, 0, c.stream, seg, pairs, live, C, Cp,
                       norms, epi);
  else if (!ta && tb)
    hipLaunchKernelGGL((k_numeric_f64<B, false, true, STAGES>), grid, block, 0, c.stream, seg, pairs, live, C, Cp,
                       norms, epi);
  else
    hipLaunchKernelGGL((k_numeric_f64<B, true, true, STAGES>), grid, block, 0, c.stream, seg, pairs, live, C, Cp,
                       norms, epi);
  LIF_HIP(hipGetLastError());
}

template <int B>
void launch_numeric_b(Ctx& c, bool ta, bool tb, const int64_t* seg, const BlockPair* pairs, int64_t nnzc,
                      const int* live, double* C, BlkOut Cp, double* norms, const Epilogue& epi, bool short_seg) {
  if (short_seg)
    launch_numeric_s<B, 1>(c, ta, tb, seg, pairs, nnzc, live, C, Cp, norms, epi);
  else
    launch_numeric_s<B, 2>(c, ta, tb, seg, pairs, nnzc, live, C, Cp, norms, epi);
}

}  // namespace

size_t symbolic_lds_bytes(int nb, bool fill) {
  const size_t nwords = (size_t)(nb + 31) / 32;
  return fill ? nwords * 8 + (size_t)nb * 4 : nwords * 4;
}

static void allow_lds(const void* fn, size_t bytes) {
  if (bytes > 48 * 1024)
    LIF_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

void launch_symbolic_count(Ctx& c, const int* arp, const int* acol, const int* brp, const int* bcol,
                           const unsigned char* diag_on, int nb, int* cnt_c, int64_t* cnt_p) {
  allow_lds((const void*)k_symbolic_count, symbolic_lds_bytes(nb, false));
  hipLaunchKernelGGL(k_symbolic_count, dim3(nb), dim3(kSymWG), symbolic_lds_bytes(nb, false), c.stream, arp, acol,
                     brp, bcol, diag_on, nb, cnt_c, cnt_p);
  LIF_HIP(hipGetLastError());
}

void launch_symbolic_fill(Ctx& c, const int* arp, const int* acol, const int* aidx, const int* brp, const int* bcol,
                          const int* bidx, BlkIn ablk, BlkIn bblk, const unsigned char* diag_on, int b, int64_t n,
                          int nb, const int* crp,
                          const int64_t* prp, int* ccol, int64_t* seg, BlockPair* pairs, unsigned char* dflag) {
  allow_lds((const void*)k_symbolic_fill, symbolic_lds_bytes(nb, true));
  hipLaunchKernelGGL(k_symbolic_fill, dim3(nb), dim3(kSymWG), symbolic_lds_bytes(nb, true), c.stream, arp, acol,
                     aidx, brp, bcol, bidx, ablk, bblk, diag_on, b, n, nb, crp, prp, ccol, seg, pairs, dflag);
  LIF_HIP(hipGetLastError());
}

void launch_numeric(Ctx& c, int prec, bool ta, bool tb, const int64_t* seg, const BlockPair* pairs,
                    int64_t nnzc, const int* live, int b, double* C, BlkOut Cp, double* norms, const Epilogue& epi,
                    bool short_seg) {
  if (nnzc == 0) return;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c.timing) {
    e0 = c.take_event();
    e1 = c.take_event();
    LIF_HIP(hipEventRecord(e0, c.stream));
  }
  if (prec != LIF_FP64)
    launch_numeric_mixed(c, prec, ta, tb, seg, pairs, nnzc, live, b, C, Cp, norms, epi);
  else if (b == 64)
    launch_numeric_b<64>(c, ta, tb, seg, pairs, nnzc, live, C, Cp, norms, epi, short_seg);
  else
    launch_numeric_b<32>(c, ta, tb, seg, pairs, nnzc, live, C, Cp, norms, epi, short_seg);
  if (c.timing) {
    LIF_HIP(hipEventRecord(e1, c.stream));
    c.ev_pending.emplace_back(e0, e1);
  }
  c.stats.gemm_launches += 1;
}

}  // namespace lif
