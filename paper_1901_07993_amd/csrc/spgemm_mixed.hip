// Numeric phase of the block-sparse product in reduced input precision with
// FP32 accumulation (the precision form of the correction products), and the
// reduced-precision copies of the operand blocks it reads.
//
// Operands are never rounded inside the product: every matrix that enters
// one carries a copy of its blocks in the input precision (FP32, or BF16
// through FP32, both rounded to nearest even), made once per matrix by
// k_make_shadow or written by the product that created the matrix.  The
// copies hold op(A)'s blocks row-major and op(B)'s blocks transposed, so
// that every MFMA fragment below is one 16-byte read of consecutive k: a
// quarter of the FP64 operand bytes for BF16, half for FP32.  The FP32
// product stages both tiles of a block product in LDS once per workgroup
// (each fragment row is read by two of its four waves) and loads the next
// pair's tiles while it multiplies; the BF16 product does the same with a
// merge step's A tile and the B tiles of the output blocks taking it.  The products of one output block accumulate in FP32 MFMA
// registers; the block is written back as FP64 with its FP64 Frobenius norm
// (and, when asked, as the transposed reduced-precision copy the next
// product reads).
//
//   FP32: v_mfma_f32_16x16x4f32; in k-block kb (16 values of k) lane group
//         g = l/16 supplies k = 16 kb + 4 g + t in step t = 0..3.
//   BF16: v_mfma_f32_16x16x32_bf16; lane group g supplies k = 32 ks + 8 g + v,
//         v = 0..7, in k-step ks.
// Fragment layouts (checked on the GPU): FP32 A lane l holds A[l%16][k of
// its group], B lane l holds B[k of its group][l%16]; BF16 A lane l holds
// A[l%16][8(l/16)+v], B lane l holds B[8(l/16)+v][l%16]; both accumulate
// D[4(l/16)+r][l%16], r = 0..3.
#include "common.h"
#include "tile_mma.h"

namespace lif {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ inline unsigned short bf16_bits_rne(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ inline int64_t xcd_remap_m(int64_t wg, int64_t total) {
  const int64_t x = wg & 7, l = wg >> 3;
  const int64_t q = total >> 3, r = total & 7;
  return x * q + (x < r ? x : r) + l;
}

// output blocks per workgroup of the BF16 product (1: one block per
// workgroup, fragments straight from global memory).  With the tiles staged
// in LDS, water-10 000's BF16 part ran at 323 / 329 / 292 / 164 TFLOP/s for
// 1, 2, 4 and 8 (8 leaves one workgroup per SIMD).
#ifndef LIF_BF16_GROUP
#define LIF_BF16_GROUP 2
#endif
constexpr int kBf16Group = LIF_BF16_GROUP;

template <int B>
struct MixCfg {
  static constexpr int WAVES = (B / 32) * (B / 32);
  static constexpr int THREADS = 64 * WAVES;
};

template <int PREC>
struct Lp;
template <>
struct Lp<LIF_MIXED_FP32> {
  typedef float T;
  __device__ static T round(double v) { return (float)v; }
};
template <>
struct Lp<LIF_MIXED_BF16> {
  typedef unsigned short T;
  __device__ static T round(double v) { return bf16_bits_rne((float)v); }
};

// The block alpha A B + gamma D (Epilogue; FP64 from the FP32 accumulators),
// its FP64 sum of squares in a fixed order, its norm and its pointer; with
// OUT_LP also its transposed reduced-precision copy and that copy's pointer.
// The values are written once the norm has decided whether (and where) the
// block is kept.
template <int B, int PREC, bool OUT_LP>
__device__ inline void epilogue(const v4f (&acc)[2][2], int rb, int cb, int l16, int kq, int lane, int wave,
                                int64_t blk, double* __restrict__ C, BlkOut Cp, double* red,
                                double* __restrict__ norms, const Epilogue& epi) {
  using Cfg = MixCfg<B>;
  typedef typename Lp<PREC>::T T;
  const double* Db = epi.dsrc ? epi.dsrc[blk] : nullptr;
  double v[2][2][4];
  double ss = 0.0;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) {
      const int col = cb + 16 * tj + l16, row0 = rb + 16 * ti + 4 * kq;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double x = epi.alpha * (double)acc[ti][tj][r];
        if (Db) x += epi.gamma * gptr(Db)[(row0 + r) * B + col];
        v[ti][tj][r] = x;
        ss += x * x;
      }
    }
  for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
  if (lane == 0) red[wave] = ss;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < Cfg::WAVES; ++w) t += red[w];
    const double nrm = sqrt(t);
    if (norms) norms[blk] = nrm;
    const int64_t s = output_slot(epi, blk, nrm);
    Cp[blk] = s >= 0 ? C + s * B * B : nullptr;
    if (OUT_LP) epi.lp_ptr[blk] = s >= 0 ? static_cast<const void*>(static_cast<T*>(epi.lp_store) + s * B * B)
                                         : nullptr;
    red[Cfg::WAVES] = __longlong_as_double(s);
  }
  __syncthreads();
  const int64_t slot = __double_as_longlong(red[Cfg::WAVES]);
  if (slot < 0) return;  // dropped: never written
  double* Cb = C + slot * B * B;
  T* Lb = OUT_LP ? static_cast<T*>(epi.lp_store) + slot * B * B : nullptr;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) {
      const int col = cb + 16 * tj + l16, row0 = rb + 16 * ti + 4 * kq;
      T lv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        Cb[(row0 + r) * B + col] = v[ti][tj][r];
        lv[r] = Lp<PREC>::round(v[ti][tj][r]);
      }
      if (OUT_LP) {  // transposed: the four rows of this lane are consecutive
        T* q = Lb + col * B + row0;
        if (PREC == LIF_MIXED_BF16) {
          const unsigned lo = (unsigned)lv[0] | ((unsigned)lv[1] << 16);
          const unsigned hi = (unsigned)lv[2] | ((unsigned)lv[3] << 16);
          *reinterpret_cast<uint2*>(q) = make_uint2(lo, hi);
        } else {
          *reinterpret_cast<float4*>(q) = make_float4(lv[0], lv[1], lv[2], lv[3]);
        }
      }
    }
}

// One workgroup per output block; pair p gives op(A)'s block row-major
// (pairs[p].a) and op(B)'s block transposed (pairs[p].b), both in the input
// precision.  Each wave computes a 32 x 32 quadrant as 2 x 2 MFMA tiles.
template <int B, bool OUT_LP>
__global__ __launch_bounds__(MixCfg<B>::THREADS) void k_numeric_bf16(const int64_t* __restrict__ seg,
                                                                     const BlockPair* __restrict__ pairs,
                                                                     const int* __restrict__ live,
                                                                     double* __restrict__ C, BlkOut Cp,
                                                                     double* __restrict__ norms, Epilogue epi) {
  constexpr int KS = B / 32;
  __shared__ double red[MixCfg<B>::WAVES + 1];  // partial sums, then the output slot
  // the grid may exceed the live output count (capacity fixed before the
  // count was known); the XCD remap runs over the live blocks only
  const int64_t nlive = live_blocks(live, epi);
  if ((int64_t)blockIdx.x >= nlive) return;
  const int64_t blk = xcd_remap_m(blockIdx.x, nlive);
  const int64_t p0 = seg[blk], p1 = seg[blk + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rb = 32 * (wave / (B / 32)), cb = 32 * (wave % (B / 32));
  const int l16 = lane & 15, kq = lane >> 4;
  v4f acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int64_t p = p0; p < p1; ++p) {
    const BlockPair pr = pairs[p];
    const unsigned short* a = reinterpret_cast<const unsigned short*>(pr.a);
    const unsigned short* bt = reinterpret_cast<const unsigned short*>(pr.b);
    v8bf af[KS][2], bf[KS][2];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int k0 = 32 * ks + 8 * kq;
        af[ks][t] = *gptr(reinterpret_cast<const v8bf*>(a + (rb + 16 * t + l16) * B + k0));
        bf[ks][t] = *gptr(reinterpret_cast<const v8bf*>(bt + (cb + 16 * t + l16) * B + k0));
      }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[ks][0], bf[ks][0], acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[ks][0], bf[ks][1], acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[ks][1], bf[ks][0], acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[ks][1], bf[ks][1], acc[1][1], 0, 0, 0);
    }
  }
  epilogue<B, LIF_MIXED_BF16, OUT_LP>(acc, rb, cb, l16, kq, lane, wave, blk, C, Cp, red, norms, epi);
}

// BF16 with operand sharing: a workgroup computes G consecutive output blocks
// (in the output's block order), walking their G lists of block products
// together.  At each step it takes the smallest A block pointer among the
// lists' next products, loads that block's fragments once, and runs the
// products of every list whose next product has that A block (an A block
// shared by several outputs of a row is read once instead of G times).  Each
// list is still consumed in its own order, with the same MFMA sequence per
// output block as k_numeric_bf16, so the blocks are bitwise the same; only
// the sharing depends on the A blocks of a row lying at increasing addresses
// (true for the input-precision copies, stored in block order).
template <int B, bool OUT_LP, int G>
__global__ __launch_bounds__(MixCfg<B>::THREADS) void k_numeric_bf16_group(const int64_t* __restrict__ seg,
                                                                           const BlockPair* __restrict__ pairs,
                                                                           const int* __restrict__ live,
                                                                           double* __restrict__ C, BlkOut Cp,
                                                                           double* __restrict__ norms,
                                                                           Epilogue epi, int64_t nblocks) {
  constexpr int KS = B / 32;
  __shared__ double red[MixCfg<B>::WAVES + 1];
  // the output blocks of the launch: *live, else all nblocks (the grid has
  // one workgroup per G of them, so it does not count them); none for a
  // voided product, whose row pointers workgroup 0 clears
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
  const int64_t e0 = xcd_remap_m(blockIdx.x, ngroups) * G;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rb = 32 * (wave / (B / 32)), cb = 32 * (wave % (B / 32));
  const int l16 = lane & 15, kq = lane >> 4;
  v4f acc[G][2][2];
  int64_t pp[G], pe[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const bool in = e0 + g < nlive;
    pp[g] = in ? seg[e0 + g] : 0;
    pe[g] = in ? seg[e0 + g + 1] : 0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[g][a][b] = v4f{0.f, 0.f, 0.f, 0.f};
  }
  // one merge step's A tile and the B tiles of the lists taking it staged in
  // LDS once per workgroup (padded rows: the 16 rows a fragment read touches
  // fall in different banks); the next step's tiles are loaded into
  // registers while the current one is multiplied
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  constexpr int LDP = B + 8;                                  // bf16 per padded row
  constexpr int NV = B * B / 8 / MixCfg<B>::THREADS;          // 16-byte pieces per thread per tile
  __shared__ __attribute__((aligned(16))) unsigned short As[B * LDP];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[G][B * LDP];
  v4u sa[NV], sb[G][NV];
  uintptr_t amin = 0, anext = 0;
  bool take[G], tnext[G];
  // the next merge step from the lists' heads: the smallest A block and the
  // lists whose head has it (uniform over the workgroup)
  auto plan = [&](uintptr_t& am, bool (&tk)[G]) {
    am = ~uintptr_t(0);
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (pp[g] < pe[g]) am = min(am, reinterpret_cast<uintptr_t>(pairs[pp[g]].a));
#pragma unroll
    for (int g = 0; g < G; ++g) tk[g] = pp[g] < pe[g] && reinterpret_cast<uintptr_t>(pairs[pp[g]].a) == am;
    return am != ~uintptr_t(0);
  };
  auto gload = [&](uintptr_t am, const bool (&tk)[G]) {
    const v4u* a = reinterpret_cast<const v4u*>(am);
#pragma unroll
    for (int v = 0; v < NV; ++v) sa[v] = *gptr(a + threadIdx.x + v * MixCfg<B>::THREADS);
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (tk[g]) {
        const v4u* bt = reinterpret_cast<const v4u*>(pairs[pp[g]].b);
#pragma unroll
        for (int v = 0; v < NV; ++v) sb[g][v] = *gptr(bt + threadIdx.x + v * MixCfg<B>::THREADS);
      }
  };
  bool have = plan(amin, take);
  if (have) gload(amin, take);
  while (have) {
    __syncthreads();  // the previous step's fragment reads are done
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int q = 8 * ((int)threadIdx.x + v * MixCfg<B>::THREADS);
      *reinterpret_cast<v4u*>(&As[(q / B) * LDP + q % B]) = sa[v];
#pragma unroll
      for (int g = 0; g < G; ++g)
        if (take[g]) *reinterpret_cast<v4u*>(&Bs[g][(q / B) * LDP + q % B]) = sb[g][v];
    }
    __syncthreads();
    v8bf af[KS][2];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int t = 0; t < 2; ++t)
        af[ks][t] = *reinterpret_cast<const v8bf*>(&As[(rb + 16 * t + l16) * LDP + 32 * ks + 8 * kq]);
    // the lists' heads advance before the next step is planned; take[]
    // still names this step's lists
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (take[g]) ++pp[g];
    const bool hn = plan(anext, tnext);
    if (hn) gload(anext, tnext);
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (take[g]) {
        v8bf bf[KS][2];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
          for (int t = 0; t < 2; ++t)
            bf[ks][t] = *reinterpret_cast<const v8bf*>(&Bs[g][(cb + 16 * t + l16) * LDP + 32 * ks + 8 * kq]);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          acc[g][0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[ks][0], bf[ks][0], acc[g][0][0], 0, 0, 0);
          acc[g][0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[ks][0], bf[ks][1], acc[g][0][1], 0, 0, 0);
          acc[g][1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[ks][1], bf[ks][0], acc[g][1][0], 0, 0, 0);
          acc[g][1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[ks][1], bf[ks][1], acc[g][1][1], 0, 0, 0);
        }
      }
    have = hn;
    amin = anext;
#pragma unroll
    for (int g = 0; g < G; ++g) take[g] = tnext[g];
  }
#pragma unroll
  for (int g = 0; g < G; ++g)
    if (e0 + g < nlive)
      epilogue<B, LIF_MIXED_BF16, OUT_LP>(acc[g], rb, cb, l16, kq, lane, wave, e0 + g, C, Cp, red, norms, epi);
}

template <int B, bool OUT_LP>
__global__ __launch_bounds__(MixCfg<B>::THREADS) void k_numeric_f32(const int64_t* __restrict__ seg,
                                                                    const BlockPair* __restrict__ pairs,
                                                                    const int* __restrict__ live,
                                                                    double* __restrict__ C, BlkOut Cp,
                                                                    double* __restrict__ norms, Epilogue epi) {
  constexpr int KB = B / 16;
  __shared__ double red[MixCfg<B>::WAVES + 1];  // partial sums, then the output slot
  const int64_t nlive = live_blocks(live, epi);
  if ((int64_t)blockIdx.x >= nlive) return;
  const int64_t blk = xcd_remap_m(blockIdx.x, nlive);
  const int64_t p0 = seg[blk], p1 = seg[blk + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rb = 32 * (wave / (B / 32)), cb = 32 * (wave % (B / 32));
  const int l16 = lane & 15, kq = lane >> 4;
  v4f acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
  // both tiles staged once per workgroup in LDS (padded rows: the 16 rows a
  // fragment read touches fall in different banks); the next pair's tiles
  // are loaded into registers while the current one is multiplied
  constexpr int LDP = B + 4;
  constexpr int NV = B * B / 4 / MixCfg<B>::THREADS;
  __shared__ __attribute__((aligned(16))) float As[B * LDP];
  __shared__ __attribute__((aligned(16))) float Bs[B * LDP];
  v4f sa[NV], sb[NV];
  auto gload = [&](int64_t p) {
    const BlockPair pr = pairs[p];
    const v4f* a = reinterpret_cast<const v4f*>(pr.a);
    const v4f* bt = reinterpret_cast<const v4f*>(pr.b);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      sa[v] = *gptr(a + threadIdx.x + v * MixCfg<B>::THREADS);
      sb[v] = *gptr(bt + threadIdx.x + v * MixCfg<B>::THREADS);
    }
  };
  if (p0 < p1) gload(p0);
  for (int64_t p = p0; p < p1; ++p) {
    if (p > p0) __syncthreads();  // the previous pair's fragment reads are done
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int q = 4 * ((int)threadIdx.x + v * MixCfg<B>::THREADS);
      *reinterpret_cast<v4f*>(&As[(q / B) * LDP + q % B]) = sa[v];
      *reinterpret_cast<v4f*>(&Bs[(q / B) * LDP + q % B]) = sb[v];
    }
    __syncthreads();
    v4f af[KB][2], bf[KB][2];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int k0 = 16 * kb + 4 * kq;
        af[kb][t] = *reinterpret_cast<const v4f*>(&As[(rb + 16 * t + l16) * LDP + k0]);
        bf[kb][t] = *reinterpret_cast<const v4f*>(&Bs[(cb + 16 * t + l16) * LDP + k0]);
      }
    if (p + 1 < p1) gload(p + 1);
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[kb][0][s], bf[kb][0][s], acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[kb][0][s], bf[kb][1][s], acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[kb][1][s], bf[kb][0][s], acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[kb][1][s], bf[kb][1][s], acc[1][1], 0, 0, 0);
      }
  }
  epilogue<B, LIF_MIXED_FP32, OUT_LP>(acc, rb, cb, l16, kq, lane, wave, blk, C, Cp, red, norms, epi);
}

// Reduced-precision copy of block e of blk (one workgroup per block, the
// first *live entries): row-major, or transposed through LDS.
template <int B, int PREC, bool TRANS>
__global__ __launch_bounds__(256) void k_make_shadow(BlkIn blk, const int* __restrict__ live,
                                                     typename Lp<PREC>::T* __restrict__ store,
                                                     const void** __restrict__ ptr) {
  typedef typename Lp<PREC>::T T;
  __shared__ T tile[TRANS ? B * (B + 1) : 1];
  const int64_t e = blockIdx.x;
  if (e >= (int64_t)*live) return;
  const double* src = blk[e];
  if (!src) {
    if (threadIdx.x == 0) ptr[e] = nullptr;
    return;
  }
  T* dst = store + e * B * B;
  const auto* s2 = gptr(reinterpret_cast<const v2d*>(src));
  for (int q = threadIdx.x; q < B * B / 2; q += 256) {
    const v2d v = s2[q];
    const int i = (2 * q) / B, j = (2 * q) % B;
    if (TRANS) {
      tile[i * (B + 1) + j] = Lp<PREC>::round(v.x);
      tile[i * (B + 1) + j + 1] = Lp<PREC>::round(v.y);
    } else {
      dst[2 * q] = Lp<PREC>::round(v.x);
      dst[2 * q + 1] = Lp<PREC>::round(v.y);
    }
  }
  if (TRANS) {
    __syncthreads();
    for (int q = threadIdx.x; q < B * B; q += 256) {
      const int j = q / B, i = q % B;  // dst row j holds column j of the block
      dst[q] = tile[i * (B + 1) + j];
    }
  }
  if (threadIdx.x == 0) ptr[e] = dst;
}

template <int B, int PREC>
void make_shadow_b(Ctx& c, bool transposed, BlkIn blk, int64_t n, const int* live, void* store,
                   const void** ptr) {
  typedef typename Lp<PREC>::T T;
  if (transposed)
    hipLaunchKernelGGL((k_make_shadow<B, PREC, true>), dim3((unsigned)n), dim3(256), 0, c.stream, blk, live,
                       static_cast<T*>(store), ptr);
  else
    hipLaunchKernelGGL((k_make_shadow<B, PREC, false>), dim3((unsigned)n), dim3(256), 0, c.stream, blk, live,
                       static_cast<T*>(store), ptr);
}

template <int B>
void launch_mixed_b(Ctx& c, int prec, const int64_t* seg, const BlockPair* pairs, int64_t nnzc, const int* live,
                    double* C, BlkOut Cp, double* norms, const Epilogue& epi) {
  const dim3 grid((unsigned)nnzc), block(MixCfg<B>::THREADS);
  const bool out_lp = epi.lp_store != nullptr;
  if (prec == LIF_MIXED_FP32) {
    if (out_lp)
      hipLaunchKernelGGL((k_numeric_f32<B, true>), grid, block, 0, c.stream, seg, pairs, live, C, Cp, norms, epi);
    else
      hipLaunchKernelGGL((k_numeric_f32<B, false>), grid, block, 0, c.stream, seg, pairs, live, C, Cp, norms, epi);
  } else if (kBf16Group > 1) {
    const dim3 ggrid((unsigned)((nnzc + kBf16Group - 1) / kBf16Group));
    if (out_lp)
      hipLaunchKernelGGL((k_numeric_bf16_group<B, true, kBf16Group>), ggrid, block, 0, c.stream, seg, pairs, live, C,
                         Cp, norms, epi, nnzc);
    else
      hipLaunchKernelGGL((k_numeric_bf16_group<B, false, kBf16Group>), ggrid, block, 0, c.stream, seg, pairs, live,
                         C, Cp, norms, epi, nnzc);
  } else {
    if (out_lp)
      hipLaunchKernelGGL((k_numeric_bf16<B, true>), grid, block, 0, c.stream, seg, pairs, live, C, Cp, norms, epi);
    else
      hipLaunchKernelGGL((k_numeric_bf16<B, false>), grid, block, 0, c.stream, seg, pairs, live, C, Cp, norms, epi);
  }
}

}  // namespace

void launch_numeric_mixed(Ctx& c, int prec, const int64_t* seg, const BlockPair* pairs, int64_t nnzc,
                          const int* live, int b, double* C, BlkOut Cp, double* norms, const Epilogue& epi) {
  LIF_REQUIRE(prec == LIF_MIXED_FP32 || prec == LIF_MIXED_BF16, LIF_ERR_INVALID, "mixed product: precision");
  if (b == 64)
    launch_mixed_b<64>(c, prec, seg, pairs, nnzc, live, C, Cp, norms, epi);
  else
    launch_mixed_b<32>(c, prec, seg, pairs, nnzc, live, C, Cp, norms, epi);
  LIF_HIP(hipGetLastError());
}

void launch_make_shadow(Ctx& c, int prec, bool transposed, BlkIn blk, int64_t n, const int* live, int b,
                        void* store, const void** ptr) {
  if (n == 0) return;
  if (prec == LIF_MIXED_FP32) {
    if (b == 64)
      make_shadow_b<64, LIF_MIXED_FP32>(c, transposed, blk, n, live, store, ptr);
    else
      make_shadow_b<32, LIF_MIXED_FP32>(c, transposed, blk, n, live, store, ptr);
  } else {
    if (b == 64)
      make_shadow_b<64, LIF_MIXED_BF16>(c, transposed, blk, n, live, store, ptr);
    else
      make_shadow_b<32, LIF_MIXED_BF16>(c, transposed, blk, n, live, store, ptr);
  }
  LIF_HIP(hipGetLastError());
}

}  // namespace lif
