// Batched leaf factorization S_leaf^{-1} = Z Z^T with Z = U^{-1} upper
// triangular, S_leaf = U^T U (Cholesky followed by triangular inversion: the
// BLAS leaf routine of Alg. 1 and Alg. 2).  All leaves of the localized
// recursion are factorized together.
//
// Storage: each leaf is a grid of nbb x nbb b x b tiles of which only the
// upper triangle (j >= i) is kept, packed row by row; tile (i, j) of leaf s
// is tile number tile0[s] + i nbb - i (i - 1) / 2 + (j - i).  In block-CSR
// terms the packed Z buffer is already the value array of the block-diagonal
// upper-triangular result, so the truncation pass reads it in place.
//
// Blocked right-looking Cholesky, one host step per tile column k:
//   potrf  U_kk = chol(S_kk) in LDS, and Z_kk = U_kk^{-1}   (one WG per leaf)
//   trsm   U_kj = Z_kk^T S_kj, j > k                          (WG per tile)
//   update S_ij -= U_ki^T U_kj, k < i <= j                    (WG per tile)
// then the inverse by tile columns j:
//   Z_ij = -(sum_{k=i}^{j-1} Z_ik U_kj) Z_jj, i < j
// Tile products run on FP64 MFMA (tile_mma.h).  Padded rows of the last
// leaf carry a unit diagonal during the factorization and are zeroed after.
// A byte per packed tile records whether the tile of S / U can be nonzero:
// tiles outside S's pattern stay zero unless an update reaches them, and
// products with a zero U tile are skipped, so a banded S costs a banded
// Cholesky (the inverse itself fills the upper triangle).
#include "common.h"
#include "tile_mma.h"

namespace lif {

namespace {

__device__ inline int64_t packed_tile(int64_t tile0, int nbb, int i, int j) {
  return tile0 + (int64_t)i * nbb - (int64_t)i * (i - 1) / 2 + (j - i);
}

__global__ __launch_bounds__(256) void k_chol_scatter(const int* __restrict__ row_of, const int* __restrict__ col,
                                                      const double* __restrict__ val, int b,
                                                      const int* __restrict__ base_of_row,
                                                      const int* __restrict__ blk0, const int* __restrict__ nbbv,
                                                      const int64_t* __restrict__ tile0, double* __restrict__ U,
                                                      unsigned char* __restrict__ nz) {
  const int64_t e = blockIdx.x;
  const int I = row_of[e], J = col[e];
  const int s = base_of_row[I];
  if (s < 0 || base_of_row[J] != s || J < I) return;
  const int i = I - blk0[s], j = J - blk0[s];
  const int64_t t = packed_tile(tile0[s], nbbv[s], i, j);
  const double2* src = reinterpret_cast<const double2*>(val + e * (int64_t)b * b);
  double2* dst = reinterpret_cast<double2*>(U + t * (int64_t)b * b);
  for (int q = threadIdx.x; q < b * b / 2; q += 256) dst[q] = src[q];
  if (threadIdx.x == 0) nz[t] = 1;
}

// set (pad = 1) or clear (pad = 0) the diagonal of padded rows of the last tile
__global__ void k_chol_pad(int nbase, const int* __restrict__ nbbv, const int* __restrict__ rowsv,
                           const int64_t* __restrict__ tile0, int b, double* __restrict__ M, double value) {
  const int s = blockIdx.x;
  const int nbb = nbbv[s];
  const int real = rowsv[s] - (nbb - 1) * b;
  const int64_t t = packed_tile(tile0[s], nbb, nbb - 1, nbb - 1);
  for (int r = real + threadIdx.x; r < b; r += blockDim.x) M[t * b * b + (int64_t)r * b + r] = value;
}

// Cholesky of the diagonal tile (k, k) and the inverse of its factor, in LDS.
// G = 256 / B threads share a column and split its dot products by residue
// of the summation index, reducing with lane shuffles (they sit in one wave).
//   rows of U, top to bottom: s_c = T[j][c] - sum_{i<j} U[i][j] U[i][c],
//     U[j][j] = sqrt(s_j), U[j][c] = s_c / U[j][j]        (2 barriers per row)
//   columns of W = U^{-1}, independently: W[c][c] = 1 / U[c][c],
//     W[r][c] = -sum_{q=r+1}^{c} U[r][q] W[q][c] / U[r][r], r = c-1 .. 0;
//     the lane owning residue r % G writes W[r][c], and each lane only reads
//     the W entries of its own residue, so no barrier is needed.
template <int B>
__global__ __launch_bounds__(256) void k_potrf(int k, const int* __restrict__ nbbv, const int* __restrict__ blk0,
                                               const int64_t* __restrict__ tile0, double* __restrict__ U,
                                               double* __restrict__ Z, int* __restrict__ err) {
  constexpr int L = B + 1;
  constexpr int G = 256 / B;
  __shared__ double T[B * L];
  __shared__ double W[B * L];
  const int s = blockIdx.x;
  const int nbb = nbbv[s];
  if (k >= nbb) return;
  const int64_t t = packed_tile(tile0[s], nbb, k, k);
  double* g = U + t * B * B;
  for (int q = threadIdx.x; q < B * B; q += 256) T[(q / B) * L + (q % B)] = g[q];
  __syncthreads();
  __shared__ double piv;
  const int c = threadIdx.x / G, gi = threadIdx.x % G;
  for (int j = 0; j < B; ++j) {
    double v = 0.0;
    if (c >= j) {
      // four independent partial sums keep several LDS reads in flight
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int i = gi;
      for (; i + 3 * G < j; i += 4 * G) {
        a0 += T[i * L + j] * T[i * L + c];
        a1 += T[(i + G) * L + j] * T[(i + G) * L + c];
        a2 += T[(i + 2 * G) * L + j] * T[(i + 2 * G) * L + c];
        a3 += T[(i + 3 * G) * L + j] * T[(i + 3 * G) * L + c];
      }
      for (; i < j; i += G) a0 += T[i * L + j] * T[i * L + c];
      double acc = (a0 + a1) + (a2 + a3);
      for (int off = 1; off < G; off <<= 1) acc += __shfl_xor(acc, off, 64);
      v = T[j * L + c] - acc;
      if (c == j && gi == 0) piv = v;
    }
    __syncthreads();  // pivot visible; every read of row j's old values done
    double d = piv;
    if (!(d > 0.0)) {
      if (threadIdx.x == 0) atomicMin(&err[s], (blk0[s] + k) * B + j);
      d = 1.0;
    }
    const double p = sqrt(d);
    if (gi == 0 && c >= j) T[j * L + c] = (c == j) ? p : v / p;
    __syncthreads();  // row j of U final before the next row reads it
  }
  for (int r = gi; r < B; r += G) W[r * L + c] = 0.0;
  // reciprocal pivots once, so the column sweeps multiply instead of divide
  __shared__ double rdiag[B];
  for (int r = threadIdx.x; r < B; r += 256) rdiag[r] = 1.0 / T[r * L + r];
  __syncthreads();
  {
    if (c % G == gi) W[c * L + c] = rdiag[c];
    for (int r = c - 1; r >= 0; --r) {
      // q in (r, c] with q % G == gi, four independent partial sums
      const int q0 = r + 1 + ((gi - (r + 1) % G) + G) % G;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int q = q0;
      for (; q + 3 * G <= c; q += 4 * G) {
        a0 += T[r * L + q] * W[q * L + c];
        a1 += T[r * L + q + G] * W[(q + G) * L + c];
        a2 += T[r * L + q + 2 * G] * W[(q + 2 * G) * L + c];
        a3 += T[r * L + q + 3 * G] * W[(q + 3 * G) * L + c];
      }
      for (; q <= c; q += G) a0 += T[r * L + q] * W[q * L + c];
      double acc = (a0 + a1) + (a2 + a3);
      for (int off = 1; off < G; off <<= 1) acc += __shfl_xor(acc, off, 64);
      if (r % G == gi) W[r * L + c] = -acc * rdiag[r];
    }
  }
  __syncthreads();
  double* gz = Z + t * B * B;
  for (int q = threadIdx.x; q < B * B; q += 256) {
    const int r = q / B, cc = q % B;
    g[q] = (cc >= r) ? T[r * L + cc] : 0.0;
    gz[q] = (cc >= r) ? W[r * L + cc] : 0.0;
  }
}

// U_kj = Z_kk^T U_kj for j = k + 1 + blockIdx.x
template <int B>
__global__ __launch_bounds__(TileCfg<B>::THREADS) void k_trsm(int k, const int* __restrict__ nbbv,
                                                              const int64_t* __restrict__ tile0,
                                                              double* __restrict__ U, const double* __restrict__ Z,
                                                              const unsigned char* __restrict__ nz) {
  using Cfg = TileCfg<B>;
  __shared__ double As[Cfg::LDS_DOUBLES];
  __shared__ double Bs[Cfg::LDS_DOUBLES];
  const int s = blockIdx.y;
  const int nbb = nbbv[s];
  const int j = k + 1 + blockIdx.x;
  if (j >= nbb || !nz[packed_tile(tile0[s], nbb, k, j)]) return;
  const Frag f = frag_coords<B>();
  v2d reg[Cfg::V2];
  tile_load<B>(Z + packed_tile(tile0[s], nbb, k, k) * B * B, reg);
  tile_store<B>(As, reg, true);  // op(A) = Z_kk^T: LDS row k is row k of Z_kk
  double* g = U + packed_tile(tile0[s], nbb, k, j) * B * B;
  tile_load<B>(g, reg);
  tile_store<B>(Bs, reg, true);
  __syncthreads();
  v4d acc[2][2];
  acc_zero(acc);
  tile_mma<B>(As, Bs, f, acc);
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) g[acc_row(f, ti, r) * B + acc_col(f, tj)] = acc[ti][tj][r];
}

__device__ inline void tri_decode(int64_t t, int& ip, int& jp) {
  // t = jp (jp + 1) / 2 + ip with 0 <= ip <= jp
  int j = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((int64_t)(j + 1) * (j + 2) / 2 <= t) ++j;
  while ((int64_t)j * (j + 1) / 2 > t) --j;
  jp = j;
  ip = (int)(t - (int64_t)j * (j + 1) / 2);
}

// U_ij -= U_ki^T U_kj for k < i <= j
template <int B>
__global__ __launch_bounds__(TileCfg<B>::THREADS) void k_update(int k, const int* __restrict__ nbbv,
                                                                const int64_t* __restrict__ tile0,
                                                                double* __restrict__ U, unsigned char* __restrict__ nz) {
  using Cfg = TileCfg<B>;
  __shared__ double As[Cfg::LDS_DOUBLES];
  __shared__ double Bs[Cfg::LDS_DOUBLES];
  const int s = blockIdx.y;
  const int nbb = nbbv[s];
  const int m = nbb - k - 1;
  const int64_t t = blockIdx.x;
  if (m <= 0 || t >= (int64_t)m * (m + 1) / 2) return;
  int ip, jp;
  tri_decode(t, ip, jp);
  const int i = k + 1 + ip, j = k + 1 + jp;
  if (!nz[packed_tile(tile0[s], nbb, k, i)] || !nz[packed_tile(tile0[s], nbb, k, j)]) return;
  const Frag f = frag_coords<B>();
  v2d reg[Cfg::V2];
  tile_load<B>(U + packed_tile(tile0[s], nbb, k, i) * B * B, reg);
  tile_store<B>(As, reg, true);  // op(A) = U_ki^T
  tile_load<B>(U + packed_tile(tile0[s], nbb, k, j) * B * B, reg);
  tile_store<B>(Bs, reg, true);
  __syncthreads();
  v4d acc[2][2];
  acc_zero(acc);
  tile_mma<B>(As, Bs, f, acc);
  double* g = U + packed_tile(tile0[s], nbb, i, j) * B * B;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int idx = acc_row(f, ti, r) * B + acc_col(f, tj);
        g[idx] -= acc[ti][tj][r];
      }
  if (threadIdx.x == 0) nz[packed_tile(tile0[s], nbb, i, j)] = 1;
}

// Z_ij = -(sum_{k=i}^{j-1} Z_ik U_kj) Z_jj for i = blockIdx.x < j
template <int B>
__global__ __launch_bounds__(TileCfg<B>::THREADS) void k_trinv(int j, const int* __restrict__ nbbv,
                                                               const int64_t* __restrict__ tile0,
                                                               const double* __restrict__ U,
                                                               double* __restrict__ Z,
                                                               const unsigned char* __restrict__ nz) {
  using Cfg = TileCfg<B>;
  __shared__ double As[Cfg::LDS_DOUBLES];
  __shared__ double Bs[Cfg::LDS_DOUBLES];
  const int s = blockIdx.y;
  const int nbb = nbbv[s];
  const int i = blockIdx.x;
  if (j >= nbb || i >= j) return;
  const Frag f = frag_coords<B>();
  const int64_t t0 = tile0[s];
  v4d acc[2][2];
  acc_zero(acc);
  v2d ra[Cfg::V2], rb[Cfg::V2];
  // k with U_kj != 0, visited in ascending order; the next pair's tiles are
  // loaded into registers while the current one is multiplied
  auto next_k = [&](int k) {
    while (k < j && !nz[packed_tile(t0, nbb, k, j)]) ++k;
    return k;
  };
  int k = next_k(i);
  if (k >= j) return;  // Z_ij = 0 (the buffer starts zeroed)
  tile_load<B>(Z + packed_tile(t0, nbb, i, k) * B * B, ra);
  tile_load<B>(U + packed_tile(t0, nbb, k, j) * B * B, rb);
  while (k < j) {
    __syncthreads();
    tile_store<B>(As, ra, false);  // op(A) = Z_ik
    tile_store<B>(Bs, rb, true);
    __syncthreads();
    const int kn = next_k(k + 1);
    if (kn < j) {
      tile_load<B>(Z + packed_tile(t0, nbb, i, kn) * B * B, ra);
      tile_load<B>(U + packed_tile(t0, nbb, kn, j) * B * B, rb);
    }
    tile_mma<B>(As, Bs, f, acc);
    k = kn;
  }
  __syncthreads();
  // W (accumulators) becomes the A operand: LDS row c holds column c of W
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) As[acc_col(f, tj) * Cfg::LD + acc_row(f, ti, r)] = acc[ti][tj][r];
  tile_load<B>(Z + packed_tile(t0, nbb, j, j) * B * B, rb);
  tile_store<B>(Bs, rb, true);
  __syncthreads();
  acc_zero(acc);
  tile_mma<B>(As, Bs, f, acc);
  double* g = Z + packed_tile(t0, nbb, i, j) * B * B;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) g[acc_row(f, ti, r) * B + acc_col(f, tj)] = -acc[ti][tj][r];
}

}  // namespace

#define LIF_LAUNCH(...)              \
  do {                               \
    hipLaunchKernelGGL(__VA_ARGS__); \
    LIF_HIP(hipGetLastError());      \
  } while (0)

void launch_chol_scatter(Ctx& c, const int* row_of, const int* col, const double* val, int64_t nnzb, int b,
                         const int* base_of_row, const int* blk0, const int* nbb, const int64_t* tile0, double* U,
                         unsigned char* nz) {
  if (nnzb == 0) return;
  LIF_LAUNCH(k_chol_scatter, dim3((unsigned)nnzb), dim3(256), 0, c.stream, row_of, col, val, b, base_of_row, blk0,
             nbb, tile0, U, nz);
}

void launch_chol_pad(Ctx& c, int nbase, const int* nbb, const int* rows, const int64_t* tile0, int b, double* M,
                     double value) {
  LIF_LAUNCH(k_chol_pad, dim3(nbase), dim3(64), 0, c.stream, nbase, nbb, rows, tile0, b, M, value);
}

void launch_potrf(Ctx& c, int k, int nbase, const int* nbb, const int* blk0, const int64_t* tile0, int b, double* U,
                  double* Z, int* err) {
  if (b == 64)
    LIF_LAUNCH(k_potrf<64>, dim3(nbase), dim3(256), 0, c.stream, k, nbb, blk0, tile0, U, Z, err);
  else
    LIF_LAUNCH(k_potrf<32>, dim3(nbase), dim3(256), 0, c.stream, k, nbb, blk0, tile0, U, Z, err);
}

void launch_trsm(Ctx& c, int k, int nbase, int max_nbb, const int* nbb, const int64_t* tile0, int b, double* U,
                 const double* Z, const unsigned char* nz) {
  if (max_nbb - k - 1 <= 0) return;
  dim3 grid(max_nbb - k - 1, nbase);
  if (b == 64)
    LIF_LAUNCH(k_trsm<64>, grid, dim3(TileCfg<64>::THREADS), 0, c.stream, k, nbb, tile0, U, Z, nz);
  else
    LIF_LAUNCH(k_trsm<32>, grid, dim3(TileCfg<32>::THREADS), 0, c.stream, k, nbb, tile0, U, Z, nz);
}

void launch_update(Ctx& c, int k, int nbase, int max_nbb, const int* nbb, const int64_t* tile0, int b, double* U,
                   unsigned char* nz) {
  const int64_t m = max_nbb - k - 1;
  if (m <= 0) return;
  dim3 grid((unsigned)(m * (m + 1) / 2), nbase);
  if (b == 64)
    LIF_LAUNCH(k_update<64>, grid, dim3(TileCfg<64>::THREADS), 0, c.stream, k, nbb, tile0, U, nz);
  else
    LIF_LAUNCH(k_update<32>, grid, dim3(TileCfg<32>::THREADS), 0, c.stream, k, nbb, tile0, U, nz);
}

void launch_trinv(Ctx& c, int j, int nbase, const int* nbb, const int64_t* tile0, int b, const double* U, double* Z,
                  const unsigned char* nz) {
  if (j <= 0) return;
  dim3 grid(j, nbase);
  if (b == 64)
    LIF_LAUNCH(k_trinv<64>, grid, dim3(TileCfg<64>::THREADS), 0, c.stream, j, nbb, tile0, U, Z, nz);
  else
    LIF_LAUNCH(k_trinv<32>, grid, dim3(TileCfg<32>::THREADS), 0, c.stream, j, nbb, tile0, U, Z, nz);
}

}  // namespace lif
