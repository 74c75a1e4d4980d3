// FP64 MFMA building blocks for b x b tile products on gfx950 (b = 32, 64).
//
// A workgroup of (b/32)^2 waves owns one b x b output tile; wave w computes
// the 32 x 32 quadrant (32 * (w / (b/32)), 32 * (w % (b/32))) as 2 x 2
// v_mfma_f64_16x16x4f64 tiles held in registers (4 doubles each per lane).
//
// Operand fragments of v_mfma_f64_16x16x4f64 (64 lanes):
//   A (16 x 4): lane l holds A[l % 16][l / 16]
//   B (4 x 16): lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l holds D[4 r + l / 16][l % 16], r = 0..3 (the FP64
//                variant spreads rows over lane groups first, unlike the
//                FP32 16x16 variants)
// Both operands are staged in LDS k-major (row k holds A[:, k] resp. B[k, :])
// so each fragment read is 16 consecutive doubles per quarter-wave.
#pragma once

#include <hip/hip_runtime.h>

namespace lif {

typedef double v4d __attribute__((ext_vector_type(4)));
// native 2-vector for the prefetch registers (HIP's double2 struct is copied
// through memory when stored whole, which sends the arrays to scratch)
typedef double v2d __attribute__((ext_vector_type(2)));

template <int B>
struct TileCfg {
  static constexpr int WAVES = (B / 32) * (B / 32);
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int LD = B + 2;                // LDS row stride in doubles
  static constexpr int V2 = B * B / 2 / THREADS;  // double2 per thread per tile
  static constexpr int LDS_DOUBLES = B * LD;
};

// Global (row-major b x b tile) -> registers, coalesced 16-byte loads.
template <int B>
__device__ __attribute__((always_inline)) inline void tile_load(const double* __restrict__ g,
                                                                v2d (&reg)[TileCfg<B>::V2]) {
  using Cfg = TileCfg<B>;
  const auto* p = gptr(reinterpret_cast<const v2d*>(g));
#pragma unroll
  for (int v = 0; v < Cfg::V2; ++v) reg[v] = p[threadIdx.x + v * Cfg::THREADS];
}

// Registers -> LDS, k-major.  `direct`: LDS row r takes global row r
// (operand used as its own k-major layout); otherwise LDS row c takes global
// column c (a transposing store).
template <int B>
__device__ __attribute__((always_inline)) inline void tile_store(double* __restrict__ s,
                                                                 const v2d (&reg)[TileCfg<B>::V2], bool direct) {
  using Cfg = TileCfg<B>;
#pragma unroll
  for (int v = 0; v < Cfg::V2; ++v) {
    const int q = 2 * (threadIdx.x + v * Cfg::THREADS);
    const int r = q / B, c = q % B;
    if (direct) {
      *reinterpret_cast<v2d*>(s + r * Cfg::LD + c) = reg[v];
    } else {
      s[c * Cfg::LD + r] = reg[v].x;
      s[(c + 1) * Cfg::LD + r] = reg[v].y;
    }
  }
}

struct Frag {
  int rb, cb, l16, kq, lane, wave;
};

template <int B>
__device__ inline Frag frag_coords() {
  Frag f;
  f.lane = threadIdx.x & 63;
  f.wave = threadIdx.x >> 6;
  f.rb = 32 * (f.wave / (B / 32));
  f.cb = 32 * (f.wave % (B / 32));
  f.l16 = f.lane & 15;
  f.kq = f.lane >> 4;
  return f;
}

__device__ inline void acc_zero(v4d (&acc)[2][2]) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
}

// acc += As^T-layout product: sum over k of A[:, k] B[k, :] for the wave's quadrant
template <int B>
__device__ inline void tile_mma(const double* __restrict__ As, const double* __restrict__ Bs, const Frag& f,
                                v4d (&acc)[2][2]) {
  using Cfg = TileCfg<B>;
#pragma unroll 4
  for (int kk = 0; kk < B / 4; ++kk) {
    const int k = 4 * kk + f.kq;
    const double a0 = As[k * Cfg::LD + f.rb + f.l16];
    const double a1 = As[k * Cfg::LD + f.rb + 16 + f.l16];
    const double b0 = Bs[k * Cfg::LD + f.cb + f.l16];
    const double b1 = Bs[k * Cfg::LD + f.cb + 16 + f.l16];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
}

// Row/column of accumulator element (ti, tj, r) of this lane.
__device__ inline int acc_row(const Frag& f, int ti, int r) { return f.rb + 16 * ti + 4 * r + f.kq; }
__device__ inline int acc_col(const Frag& f, int tj) { return f.cb + 16 * tj + f.l16; }

}  // namespace lif
