// Numeric phase of the block-sparse product in reduced input precision with
// FP32 accumulation (the precision form of the correction products): the
// FP64 operand blocks are rounded while they are staged into LDS, the
// products of one output block accumulate in FP32 MFMA registers, and the
// block is written back as FP64 together with its FP64 Frobenius norm.
//
//   FP32:  inputs rounded to FP32 (round to nearest even), v_mfma_f32_16x16x4f32,
//          operands k-major in LDS as in the FP64 kernel.
//   BF16:  inputs rounded FP64 -> FP32 -> BF16 (both round to nearest even),
//          v_mfma_f32_16x16x32_bf16; A staged row-major (row i holds A[i][k],
//          k contiguous) and B column-major (row j holds B[k][j] over k), so
//          each lane's 8 consecutive k values are one 16-byte LDS read.
// Fragment layouts (checked on the GPU): FP32 A lane l holds A[l%16][l/16],
// B lane l holds B[l/16][l%16]; BF16 A lane l holds A[l%16][8(l/16)+v],
// B lane l holds B[8(l/16)+v][l%16], v = 0..7; both accumulate
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

template <int B>
struct MixCfg {
  static constexpr int WAVES = (B / 32) * (B / 32);
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int V2 = B * B / 2 / THREADS;
  static constexpr int LDF = B + 4;   // FP32 LDS row stride (floats)
  static constexpr int LDH = B + 8;   // BF16 LDS row stride (halves), rows 16-byte aligned
};

// FP32 staging, k-major: direct -> LDS row r holds global row r.
template <int B>
__device__ inline void store_f32(float* __restrict__ s, const v2d* reg, bool direct) {
  using Cfg = MixCfg<B>;
#pragma unroll
  for (int v = 0; v < Cfg::V2; ++v) {
    const int q = 2 * (threadIdx.x + v * Cfg::THREADS);
    const int r = q / B, c = q % B;
    const float x = (float)reg[v].x, y = (float)reg[v].y;
    if (direct) {
      *reinterpret_cast<float2*>(s + r * Cfg::LDF + c) = make_float2(x, y);
    } else {
      s[c * Cfg::LDF + r] = x;
      s[(c + 1) * Cfg::LDF + r] = y;
    }
  }
}

// BF16 staging: direct -> LDS row r holds global row r, else row c holds column c.
template <int B>
__device__ inline void store_bf16(unsigned short* __restrict__ s, const v2d* reg, bool direct) {
  using Cfg = MixCfg<B>;
#pragma unroll
  for (int v = 0; v < Cfg::V2; ++v) {
    const int q = 2 * (threadIdx.x + v * Cfg::THREADS);
    const int r = q / B, c = q % B;
    const unsigned short x = bf16_bits_rne((float)reg[v].x), y = bf16_bits_rne((float)reg[v].y);
    if (direct) {
      *reinterpret_cast<unsigned*>(s + r * Cfg::LDH + c) = (unsigned)x | ((unsigned)y << 16);
    } else {
      s[c * Cfg::LDH + r] = x;
      s[(c + 1) * Cfg::LDH + r] = y;
    }
  }
}

// The block alpha A B + gamma D (Epilogue; FP64 from the FP32 accumulators),
// its FP64 sum of squares in a fixed order, its norm and its pointer.
template <int B>
__device__ inline void epilogue(const v4f (&acc)[2][2], int rb, int cb, int l16, int kq, int lane, int wave,
                                int64_t blk, double* __restrict__ C, BlkOut Cp, double* red,
                                double* __restrict__ norms, const Epilogue& epi) {
  using Cfg = MixCfg<B>;
  const double* Db = epi.dsrc ? epi.dsrc[blk] : nullptr;
  double* Cb = C + blk * B * B;
  double ss = 0.0;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int idx = (rb + 16 * ti + 4 * kq + r) * B + cb + 16 * tj + l16;
        double v = epi.alpha * (double)acc[ti][tj][r];
        if (Db) v += epi.gamma * gptr(Db)[idx];
        Cb[idx] = v;
        ss += v * v;
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
    Cp[blk] = (epi.drop && !(nrm >= epi.tau)) ? nullptr : Cb;
  }
}

template <int B, bool TA, bool TB>
__global__ __launch_bounds__(MixCfg<B>::THREADS) void k_numeric_f32(
                                                                    const int64_t* __restrict__ seg,
                                                                    const BlockPair* __restrict__ pairs,
                                                                    const int* __restrict__ live,
                                                                    double* __restrict__ C, BlkOut Cp,
                                                                    double* __restrict__ norms, Epilogue epi) {
  using Cfg = MixCfg<B>;
  __shared__ float As[B * Cfg::LDF];
  __shared__ float Bs[B * Cfg::LDF];
  __shared__ double red[Cfg::WAVES];
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
  v2d ra[Cfg::V2], rbv[Cfg::V2];
  if (p1 > p0) {  // a diagonal block of a fused identity term may have no products
    const BlockPair pr = pairs[p0];
    tile_load<B>(pr.a, ra);
    tile_load<B>(pr.b, rbv);
  }
  for (int64_t p = p0; p < p1; ++p) {
    __syncthreads();
    store_f32<B>(As, ra, TA);    // As[k][i] = op(A)[i][k]
    store_f32<B>(Bs, rbv, !TB);  // Bs[k][j] = op(B)[k][j]
    __syncthreads();
    if (p + 1 < p1) {
      const BlockPair pr = pairs[p + 1];
      tile_load<B>(pr.a, ra);
      tile_load<B>(pr.b, rbv);
    }
#pragma unroll 4
    for (int kk = 0; kk < B / 4; ++kk) {
      const int k = 4 * kk + kq;
      const float a0 = As[k * Cfg::LDF + rb + l16];
      const float a1 = As[k * Cfg::LDF + rb + 16 + l16];
      const float b0 = Bs[k * Cfg::LDF + cb + l16];
      const float b1 = Bs[k * Cfg::LDF + cb + 16 + l16];
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
    }
  }
  epilogue<B>(acc, rb, cb, l16, kq, lane, wave, blk, C, Cp, red, norms, epi);
}

template <int B, bool TA, bool TB>
__global__ __launch_bounds__(MixCfg<B>::THREADS) void k_numeric_bf16(
                                                                     const int64_t* __restrict__ seg,
                                                                     const BlockPair* __restrict__ pairs,
                                                                     const int* __restrict__ live,
                                                                     double* __restrict__ C, BlkOut Cp,
                                                                     double* __restrict__ norms, Epilogue epi) {
  using Cfg = MixCfg<B>;
  __shared__ __attribute__((aligned(16))) unsigned short As[B * Cfg::LDH];  // As[i][k]
  __shared__ __attribute__((aligned(16))) unsigned short Bs[B * Cfg::LDH];  // Bs[j][k]
  __shared__ double red[Cfg::WAVES];
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
  v2d ra[Cfg::V2], rbv[Cfg::V2];
  if (p1 > p0) {  // a diagonal block of a fused identity term may have no products
    const BlockPair pr = pairs[p0];
    tile_load<B>(pr.a, ra);
    tile_load<B>(pr.b, rbv);
  }
  for (int64_t p = p0; p < p1; ++p) {
    __syncthreads();
    store_bf16<B>(As, ra, !TA);  // As[i][k] = op(A)[i][k]
    store_bf16<B>(Bs, rbv, TB);  // Bs[j][k] = op(B)[k][j]
    __syncthreads();
    if (p + 1 < p1) {
      const BlockPair pr = pairs[p + 1];
      tile_load<B>(pr.a, ra);
      tile_load<B>(pr.b, rbv);
    }
#pragma unroll
    for (int kk = 0; kk < B / 32; ++kk) {
      const int k0 = 32 * kk + 8 * kq;
      const v8bf a0 = *reinterpret_cast<const v8bf*>(As + (rb + l16) * Cfg::LDH + k0);
      const v8bf a1 = *reinterpret_cast<const v8bf*>(As + (rb + 16 + l16) * Cfg::LDH + k0);
      const v8bf b0 = *reinterpret_cast<const v8bf*>(Bs + (cb + l16) * Cfg::LDH + k0);
      const v8bf b1 = *reinterpret_cast<const v8bf*>(Bs + (cb + 16 + l16) * Cfg::LDH + k0);
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[1][1], 0, 0, 0);
    }
  }
  epilogue<B>(acc, rb, cb, l16, kq, lane, wave, blk, C, Cp, red, norms, epi);
}

#define LIF_MIXED_DISPATCH(KERNEL, B)                                                                      \
  do {                                                                                                     \
    dim3 grid((unsigned)nnzc), block(MixCfg<B>::THREADS);                                                  \
    if (!ta && !tb)                                                                                        \
      hipLaunchKernelGGL((KERNEL<B, false, false>), grid, block, 0, c.stream, seg, pairs, live, C, Cp, norms, epi); \
    else if (ta && !tb)                                                                                    \
      hipLaunchKernelGGL((KERNEL<B, true, false>), grid, block, 0, c.stream, seg, pairs, live, C, Cp, norms, epi); \
    else if (!ta && tb)                                                                                    \
      hipLaunchKernelGGL((KERNEL<B, false, true>), grid, block, 0, c.stream, seg, pairs, live, C, Cp, norms, epi); \
    else                                                                                                   \
      hipLaunchKernelGGL((KERNEL<B, true, true>), grid, block, 0, c.stream, seg, pairs, live, C, Cp, norms, epi); \
  } while (0)

}  // namespace

void launch_numeric_mixed(Ctx& c, int prec, bool ta, bool tb, const int64_t* seg,
                          const BlockPair* pairs, int64_t nnzc, const int* live, int b, double* C, BlkOut Cp, double* norms,
                          const Epilogue& epi) {
  if (prec == LIF_MIXED_FP32) {
    if (b == 64)
      LIF_MIXED_DISPATCH(k_numeric_f32, 64);
    else
      LIF_MIXED_DISPATCH(k_numeric_f32, 32);
  } else {
    if (b == 64)
      LIF_MIXED_DISPATCH(k_numeric_bf16, 64);
    else
      LIF_MIXED_DISPATCH(k_numeric_bf16, 32);
  }
  LIF_HIP(hipGetLastError());
}

}  // namespace lif
