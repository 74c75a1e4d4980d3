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
//          and V_ik = U_ik Z_kk, i < k, in place of U_ik (no later step
//          reads U_ik)
//   update S_ij -= U_ki^T U_kj, k < i <= j                    (WG per tile)
// then the inverse by tile columns j:
//   Z_ij = -(sum_{k=i}^{j-1} Z_ik U_kj) Z_jj = -sum_{k=i}^{j-1} Z_ik V_kj, i < j
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
                                                      BlkIn val, int b,
                                                      const int* __restrict__ base_of_row,
                                                      const int* __restrict__ blk0, const int* __restrict__ nbbv,
                                                      const int64_t* __restrict__ tile0, double* __restrict__ U,
                                                      unsigned char* __restrict__ nz, int* __restrict__ band) {
  const int64_t e = blockIdx.x;
  const int I = row_of[e], J = col[e];
  const int s = base_of_row[I];
  if (s < 0 || base_of_row[J] != s || J < I) return;
  const int i = I - blk0[s], j = J - blk0[s];
  const int64_t t = packed_tile(tile0[s], nbbv[s], i, j);
  const auto* src = gptr(reinterpret_cast<const v2d*>(val[e]));
  v2d* dst = reinterpret_cast<v2d*>(U + t * (int64_t)b * b);
  v2d r[8];  // b * b / 2 / 256 <= 8 pairs per thread, all loads issued first
#pragma unroll
  for (int v = 0; v < 8; ++v)
    if (threadIdx.x + v * 256 < b * b / 2) r[v] = src[threadIdx.x + v * 256];
#pragma unroll
  for (int v = 0; v < 8; ++v)
    if (threadIdx.x + v * 256 < b * b / 2) dst[threadIdx.x + v * 256] = r[v];
  if (threadIdx.x == 0) {
    nz[t] = 1;
    atomicMax(band, j - i);
  }
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

// Lane `src`'s value of v, for every lane (two v_readlane_b32; src uniform).
__device__ __attribute__((always_inline)) inline double bcast(double v, int src) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffull), src);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), src);
  return __hiloint2double(hi, lo);
}

// 1 / sqrt(x) to full FP64 precision: the hardware estimate and two Newton
// steps y <- y + y (1 - x y^2) / 2.
__device__ __attribute__((always_inline)) inline double rsqrt_fp64(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// Orders the LDS accesses of one wavefront (the hardware keeps them in
// order; this keeps the compiler from moving them across each other).
__device__ __attribute__((always_inline)) inline void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Cholesky of the diagonal tile (k, k) and the inverse of its factor, in LDS,
// blocked by 16 x 16 sub-blocks (NS = B / 16 of them per side).  For each
// sub-block column p:
//   A (wave 0, in registers; lane c owns column c of the sub-block)
//       U_pp = chol(T_pp) by rank-1 updates: the pivot comes by v_readlane,
//       row j of U is broadcast through 16 doubles of LDS; then
//       V_pp = U_pp^{-1} by back substitution, rows of U read from LDS
//   B (one wave per task, 16x16x16 MFMA products)
//       panel  U_pq = V_pp^T T_pq, q > p
//       inverse W_rp = -Y_r V_pp, r < p
//   C (one wave per task)
//       trailing T_qq' -= U_pq^T U_pq', p < q <= q'
//       Y_r = sum_{s=r..p} W_rs U_s,p+1 for the next column's inverse blocks
// W = U^{-1} is built column block by column block from
//   W_rp = -(sum_{s=r}^{p-1} W_rs U_sp) V_pp,
// so the inverse costs no extra step.  Three barriers per sub-block column.
// NT threads (a multiple of 64) run it; LDS layout in PotrfLds.
template <int B>
struct PotrfLds {
  static constexpr int L = B + 1;
  static constexpr int NS = B / 16;
  static constexpr int YL = 17;
  static constexpr int T_OFF = 0;
  static constexpr int W_OFF = B * L;
  static constexpr int Y_OFF = 2 * B * L;
  static constexpr int R_OFF = (Y_OFF + NS * 16 * YL + 1) / 2 * 2;  // 16-byte aligned
  static constexpr int DOUBLES = R_OFF + 16;
};

// T <- the tile at g (zeros when `have` is false: a diagonal tile S does not
// have, which then fails as not positive definite)
template <int B, int NT>
__device__ __attribute__((always_inline)) inline void potrf_load(double* smem, const double* g, bool have) {
  using Lay = PotrfLds<B>;
  constexpr int NV = B * B / 2 / NT;
  double* T = smem + Lay::T_OFF;
  v2d r[NV];
  const v2d* gv = reinterpret_cast<const v2d*>(g);
#pragma unroll
  for (int v = 0; v < NV; ++v) r[v] = have ? gv[threadIdx.x + v * NT] : v2d{0.0, 0.0};
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int q = 2 * (threadIdx.x + v * NT);
    T[(q / B) * Lay::L + (q % B)] = r[v].x;
    T[(q / B) * Lay::L + (q % B) + 1] = r[v].y;
  }
}

// Factorizes T (in LDS, complete and visible to all threads) and writes U_kk
// to g, Z_kk to gz; the first non-positive pivot is reported as global row
// row0 + its index.
template <int B, int NT>
__device__ __attribute__((always_inline)) inline void potrf_tile(double* smem, double* __restrict__ g, double* __restrict__ gz, int row0,
                           int* __restrict__ err_slot) {
  using Lay = PotrfLds<B>;
  constexpr int L = Lay::L;
  constexpr int NS = Lay::NS;
  constexpr int YL = Lay::YL;
  constexpr int NW = NT / 64;
  double* T = smem + Lay::T_OFF;
  double* W = smem + Lay::W_OFF;
  double* Y = smem + Lay::Y_OFF;
  double* rowbuf = smem + Lay::R_OFF;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  int bad = -1;  // first non-positive pivot (wave 0)
  for (int p = 0; p < NS; ++p) {
    const int o = 16 * p;
    if (wave == 0) {
      double a[16], rd[16], v[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) a[i] = T[(o + i) * L + o + l16];
      // the next pivot is lane j+1's own diagonal entry less x^2: it is
      // formed before the row broadcast, keeping the broadcast off the
      // serial pivot chain
      double piv_next = bcast(a[0], 0);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        double piv = piv_next;
        if (!(piv > 0.0)) {
          if (bad < 0) bad = o + j;
          piv = 1.0;
        }
        const double rj = rsqrt_fp64(piv);
        rd[j] = rj;
        // row j of U: U[j][c] = a[j] / p_j (c > j), p_j at c = j, 0 below
        const double x = (l16 == j) ? piv * rj : (l16 > j ? a[j] * rj : 0.0);
        a[j] = x;
        if (j < 15) piv_next = bcast(fma(-x, x, a[j + 1]), j + 1);
        if (j < 15) {
          rowbuf[l16] = x;
          wave_lds_fence();
          double u[16];
#pragma unroll
          for (int i = j + 1; i < 16; ++i) u[i] = rowbuf[i];
          wave_lds_fence();  // the reads are done before the next row is written
#pragma unroll
          for (int i = j + 1; i < 16; ++i) a[i] = fma(-u[i], x, a[i]);
        }
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) a[i] = (i <= l16) ? a[i] : 0.0;
      if (lane < 16) {
#pragma unroll
        for (int i = 0; i < 16; ++i) T[(o + i) * L + o + l16] = a[i];
      }
      wave_lds_fence();
      // column c of V: V[r][c] = (delta_rc - sum_{q>r} U[r][q] V[q][c]) / U[r][r]
#pragma unroll
      for (int r = 15; r >= 0; --r) {
        double acc = (l16 == r) ? 1.0 : 0.0;
#pragma unroll
        for (int q = r + 1; q < 16; ++q) acc = fma(-T[(o + r) * L + o + q], v[q], acc);
        v[r] = acc * rd[r];
      }
      if (lane < 16) {
#pragma unroll
        for (int i = 0; i < 16; ++i) W[(o + i) * L + o + l16] = v[i];
      }
    }
    __syncthreads();
    // B: task w < NS - 1 - p is the panel block q = p + 1 + w, the others the
    // inverse blocks r = w - (NS - 1 - p); each task reads only what it writes
    // and sub-blocks no other task touches in this phase
    if (wave < NS - 1) {
      v4d acc = {0.0, 0.0, 0.0, 0.0};
      const int npanel = NS - 1 - p;
      if (wave < npanel) {
        const int q = p + 1 + wave;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const int kk = o + 4 * ks + kq;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(W[kk * L + o + l16], T[kk * L + 16 * q + l16], acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) T[(o + 4 * r + kq) * L + 16 * q + l16] = acc[r];
      } else {
        const int rb = wave - npanel;
        const double* Yr = Y + rb * 16 * YL;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const int kk = 4 * ks + kq;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Yr[l16 * YL + kk], W[(o + kk) * L + o + l16], acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) W[(16 * rb + 4 * r + kq) * L + o + l16] = -acc[r];
      }
    }
    __syncthreads();
    if (p == NS - 1) break;
    // C: trailing blocks (q1, q2), p < q1 <= q2, then the Y blocks r = 0..p
    const int m = NS - 1 - p;
    const int ntrail = m * (m + 1) / 2;
    for (int task = wave; task < ntrail + p + 1; task += NW) {
      v4d acc = {0.0, 0.0, 0.0, 0.0};
      if (task < ntrail) {
        int q1 = 0, rem = task;
        while (rem >= m - q1) {
          rem -= m - q1;
          ++q1;
        }
        const int c1 = 16 * (p + 1 + q1), c2 = c1 + 16 * rem;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const int kk = o + 4 * ks + kq;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(T[kk * L + c1 + l16], T[kk * L + c2 + l16], acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) T[(c1 + 4 * r + kq) * L + c2 + l16] -= acc[r];
      } else {
        const int rb = task - ntrail;
        const int c2 = 16 * (p + 1);
        for (int ks = 0; ks < 4 * (p + 1 - rb); ++ks) {
          const int kk = 16 * rb + 4 * ks + kq;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(W[(16 * rb + l16) * L + kk], T[kk * L + c2 + l16], acc, 0, 0,
                                                     0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) Y[rb * 16 * YL + (4 * r + kq) * YL + l16] = acc[r];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && bad >= 0) atomicMin(err_slot, row0 + bad);
#pragma unroll
  for (int v = 0; v < B * B / 2 / NT; ++v) {
    const int q = 2 * (threadIdx.x + v * NT), r = q / B, cc = q % B;
    reinterpret_cast<v2d*>(g)[q / 2] = v2d{(cc >= r) ? T[r * L + cc] : 0.0, (cc + 1 >= r) ? T[r * L + cc + 1] : 0.0};
    reinterpret_cast<v2d*>(gz)[q / 2] =
        v2d{(cc >= r) ? W[r * L + cc] : 0.0, (cc + 1 >= r) ? W[r * L + cc + 1] : 0.0};
  }
}


// Step k's diagonal tile, one workgroup per leaf (the first step; later
// steps run inside the update kernel of the step before).
template <int B>
__global__ __launch_bounds__(TileCfg<B>::THREADS) void k_potrf(int k, const int* __restrict__ nbbv,
                                                               const int* __restrict__ blk0,
                                                               const int64_t* __restrict__ tile0,
                                                               double* __restrict__ U, double* __restrict__ Z,
                                                               const unsigned char* __restrict__ nz,
                                                               int* __restrict__ err) {
  constexpr int NT = TileCfg<B>::THREADS;
  __shared__ __attribute__((aligned(16))) double smem[PotrfLds<B>::DOUBLES];
  const int s = blockIdx.x;
  const int nbb = nbbv[s];
  if (k >= nbb) return;
  const int64_t t = packed_tile(tile0[s], nbb, k, k);
  potrf_load<B, NT>(smem, U + t * B * B, nz[t] != 0);
  __syncthreads();
  potrf_tile<B, NT>(smem, U + t * B * B, Z + t * B * B, (blk0[s] + k) * B, &err[s]);
}

__device__ inline void tri_decode(int64_t t, int& ip, int& jp) {
  // t = jp (jp + 1) / 2 + ip with 0 <= ip <= jp
  int j = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((int64_t)(j + 1) * (j + 2) / 2 <= t) ++j;
  while ((int64_t)j * (j + 1) / 2 > t) --j;
  jp = j;
  ip = (int)(t - (int64_t)j * (j + 1) / 2);
}

// Registers of an MFMA accumulator -> LDS tile (row-major, stride LD), as
// an operand for tile_mma: row r of the stored tile is LDS row r.
template <int B>
__device__ __attribute__((always_inline)) inline void acc_to_lds(double* s, const v4d (&acc)[2][2], const Frag& f) {
  constexpr int LD = TileCfg<B>::LD;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) s[acc_row(f, ti, r) * LD + acc_col(f, tj)] = acc[ti][tj][r];
}

// Step k of the batched leaf factorization, one launch (grid.y = leaf).
// Task t < nupd is the trailing tile (i, j) = (k+1+ip, k+1+jp), ip <= jp,
// of the tile band:
//     U_ki = Z_kk^T T_ki and U_kj = Z_kk^T T_kj (the row-k panel of the
//     factor, recomputed by each task that needs it, so that no task waits
//     for another), then T_ij -= U_ki^T U_kj.
//   A diagonal task (i = j) also stores U_kj, in Z's (k, j) slot: Z_kj is
//   written only by the inverse's column j, after the V task of step j has
//   read U_kj there.  Task 0 -- tile (k+1, k+1), whose last update this is
//   -- then factorizes that tile in LDS (U_{k+1,k+1}, Z_{k+1,k+1}).
// The other tasks are the V tiles of column k:
//     V_ik = U_ik Z_kk for max(0, k - band) <= i < k,
//   U_ik read from Z's (i, k) slot and V_ik written to U's (i, k) slot,
//   whose T_ik no step reads any more.
// Within a step no task reads what another writes; the serial chain per
// tile column is this one launch.
template <int B>
__global__ __launch_bounds__(TileCfg<B>::THREADS) void k_step(int k, int band, int nupd, int ntask, int nbase,
                                                              const int* __restrict__ nbbv,
                                                              const int* __restrict__ blk0,
                                                              const int64_t* __restrict__ tile0,
                                                              double* __restrict__ U, double* __restrict__ Z,
                                                              unsigned char* __restrict__ nz,
                                                              int* __restrict__ err) {
  using Cfg = TileCfg<B>;
  constexpr int NT = Cfg::THREADS;
  constexpr int SMEM = (2 * Cfg::LDS_DOUBLES > PotrfLds<B>::DOUBLES) ? 2 * Cfg::LDS_DOUBLES : PotrfLds<B>::DOUBLES;
  __shared__ __attribute__((aligned(16))) double smem[SMEM];
  double* As = smem;
  double* Bs = smem + Cfg::LDS_DOUBLES;
  // 1-D grid: the first nbase workgroups are task 0 of every leaf -- the
  // serial chain -- so that they are dispatched before anything else
  int s, t;
  if ((int)blockIdx.x < nbase) {
    s = blockIdx.x;
    t = 0;
  } else {
    const int w = (int)blockIdx.x - nbase;
    s = w / (ntask - 1);
    t = 1 + w % (ntask - 1);
  }
  const int nbb = nbbv[s];
  if (k >= nbb) return;
  const int64_t t0 = tile0[s];
  const Frag f = frag_coords<B>();
  const double* zkk = Z + packed_tile(t0, nbb, k, k) * B * B;

  if (t >= nupd) {  // V task
    const int i = max(0, k - band) + (t - nupd);
    if (i >= k || !nz[packed_tile(t0, nbb, i, k)]) return;
    const int64_t tik = packed_tile(t0, nbb, i, k);
    v2d reg[Cfg::V2];
    tile_load<B>(Z + tik * B * B, reg);
    tile_store<B>(As, reg, false);  // op(A) = U_ik: LDS row c is column c of U_ik
    tile_load<B>(zkk, reg);
    tile_store<B>(Bs, reg, true);
    __syncthreads();
    v4d acc[2][2];
    acc_zero(acc);
    tile_mma<B>(As, Bs, f, acc);
    double* g = U + tik * B * B;
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r) g[acc_row(f, ti, r) * B + acc_col(f, tj)] = acc[ti][tj][r];
    return;
  }

  const int m = min(band, nbb - k - 1);
  if (t >= m * (m + 1) / 2) return;  // this leaf's band is narrower here
  int ip = 0, jp = 0;
  tri_decode(t, ip, jp);
  const int i = k + 1 + ip, j = k + 1 + jp;
  const bool diag = i == j;
  const bool next_diag = t == 0;  // tile (k+1, k+1)
  const int64_t tki = packed_tile(t0, nbb, k, i), tkj = packed_tile(t0, nbb, k, j);
  const int64_t tij = packed_tile(t0, nbb, i, j);
  double* g = U + tij * B * B;
  if (nz[tki] && nz[tkj]) {
    // a tile outside S's pattern that no earlier step reached holds no data
    // yet (the buffer is not cleared): its first update writes -acc
    const bool first = !nz[tij];
    double old[2][2][4];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r) old[ti][tj][r] = first ? 0.0 : g[acc_row(f, ti, r) * B + acc_col(f, tj)];
    v2d rz[Cfg::V2], ri[Cfg::V2], rj[Cfg::V2];
    tile_load<B>(zkk, rz);
    tile_load<B>(U + tki * B * B, ri);
    if (!diag) tile_load<B>(U + tkj * B * B, rj);
    tile_store<B>(As, rz, true);  // op(A) = Z_kk^T
    tile_store<B>(Bs, ri, true);  // op(B) = T_ki
    __syncthreads();
    v4d ui[2][2], uj[2][2];
    acc_zero(ui);
    tile_mma<B>(As, Bs, f, ui);  // U_ki
    if (!diag) {
      __syncthreads();
      tile_store<B>(Bs, rj, true);  // op(B) = T_kj
      __syncthreads();
      acc_zero(uj);
      tile_mma<B>(As, Bs, f, uj);  // U_kj
    }
    __syncthreads();
    acc_to_lds<B>(As, ui, f);  // op(A) = U_ki^T: LDS row r is row r of U_ki
    if (diag)
      acc_to_lds<B>(Bs, ui, f);
    else
      acc_to_lds<B>(Bs, uj, f);
    if (diag) {  // the panel tile for the V task of step j
      double* zs = Z + tkj * B * B;
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
          for (int r = 0; r < 4; ++r) zs[acc_row(f, ti, r) * B + acc_col(f, tj)] = ui[ti][tj][r];
    }
    __syncthreads();
    v4d acc[2][2];
    acc_zero(acc);
    tile_mma<B>(As, Bs, f, acc);
    __syncthreads();  // every fragment read and flag read done: LDS and nz may change
    if (next_diag) {
      double* T = smem + PotrfLds<B>::T_OFF;
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            T[acc_row(f, ti, r) * PotrfLds<B>::L + acc_col(f, tj)] = old[ti][tj][r] - acc[ti][tj][r];
    } else {
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
          for (int r = 0; r < 4; ++r) g[acc_row(f, ti, r) * B + acc_col(f, tj)] = old[ti][tj][r] - acc[ti][tj][r];
    }
    if (threadIdx.x == 0) nz[tij] = 1;
  } else if (next_diag) {
    potrf_load<B, NT>(smem, g, nz[tij] != 0);
  }
  if (next_diag) {
    __syncthreads();
    potrf_tile<B, NT>(smem, g, Z + tij * B * B, (blk0[s] + k + 1) * B, &err[s]);
  }
}

// Tile columns j0 .. j0 + ncol - 1 of the inverse, one workgroup per
// (row i, leaf): Z_ij = -sum_{k=i}^{j-1} Z_ik V_kj for every column j > i of
// the range, V_kj = U_kj Z_jj (held in U's place), V_kj = 0 for k < j -
// band.  A row's columns are done in order by the same workgroup (column j+1
// reads the Z_ij it just wrote), so the tiles Z_ik two neighbouring columns
// share are read from HBM once and then found in L2.
template <int B>
__global__ __launch_bounds__(TileCfg<B>::THREADS) void k_trinv(int j0, int ncol, int band,
                                                               const int* __restrict__ nbbv,
                                                               const int64_t* __restrict__ tile0,
                                                               const double* __restrict__ V,
                                                               double* __restrict__ Z,
                                                               const unsigned char* __restrict__ nz) {
  using Cfg = TileCfg<B>;
  __shared__ double As[Cfg::LDS_DOUBLES];
  __shared__ double Bs[Cfg::LDS_DOUBLES];
  const int s = blockIdx.y;
  const int nbb = nbbv[s];
  const int i = blockIdx.x;
  const Frag f = frag_coords<B>();
  const int64_t t0 = tile0[s];
  for (int j = max(j0, i + 1); j < j0 + ncol && j < nbb; ++j) {
    __syncthreads();  // the previous column's LDS reads and Z writes are done
    v4d acc[2][2];
    acc_zero(acc);
    v2d ra[Cfg::V2], rb[Cfg::V2];
    // k with V_kj != 0, visited in ascending order; the next pair's tiles are
    // loaded into registers while the current one is multiplied
    auto next_k = [&](int k) {
      while (k < j && !nz[packed_tile(t0, nbb, k, j)]) ++k;
      return k;
    };
    int k = next_k(max(i, j - band));
    if (k >= j) {  // Z_ij = 0 (the buffer is not cleared beforehand)
      v2d* g = reinterpret_cast<v2d*>(Z + packed_tile(t0, nbb, i, j) * B * B);
#pragma unroll
      for (int v = 0; v < Cfg::V2; ++v) g[threadIdx.x + v * Cfg::THREADS] = v2d{0.0, 0.0};
      continue;
    }
    tile_load<B>(Z + packed_tile(t0, nbb, i, k) * B * B, ra);
    tile_load<B>(V + packed_tile(t0, nbb, k, j) * B * B, rb);
    bool first = true;
    while (k < j) {
      if (!first) __syncthreads();
      first = false;
      tile_store<B>(As, ra, false);  // op(A) = Z_ik
      tile_store<B>(Bs, rb, true);
      __syncthreads();
      const int kn = next_k(k + 1);
      if (kn < j) {
        tile_load<B>(Z + packed_tile(t0, nbb, i, kn) * B * B, ra);
        tile_load<B>(V + packed_tile(t0, nbb, kn, j) * B * B, rb);
      }
      tile_mma<B>(As, Bs, f, acc);
      k = kn;
    }
    double* g = Z + packed_tile(t0, nbb, i, j) * B * B;
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r) g[acc_row(f, ti, r) * B + acc_col(f, tj)] = -acc[ti][tj][r];
  }
}

}  // namespace

#define LIF_LAUNCH(...)              \
  do {                               \
    hipLaunchKernelGGL(__VA_ARGS__); \
    LIF_HIP(hipGetLastError());      \
  } while (0)

void launch_chol_scatter(Ctx& c, const int* row_of, const int* col, BlkIn val, int64_t nnzb, int b,
                         const int* base_of_row, const int* blk0, const int* nbb, const int64_t* tile0, double* U,
                         unsigned char* nz, int* band) {
  if (nnzb == 0) return;
  LIF_LAUNCH(k_chol_scatter, dim3((unsigned)nnzb), dim3(256), 0, c.stream, row_of, col, val, b, base_of_row, blk0,
             nbb, tile0, U, nz, band);
}

void launch_chol_pad(Ctx& c, int nbase, const int* nbb, const int* rows, const int64_t* tile0, int b, double* M,
                     double value) {
  LIF_LAUNCH(k_chol_pad, dim3(nbase), dim3(64), 0, c.stream, nbase, nbb, rows, tile0, b, M, value);
}

void launch_potrf(Ctx& c, int k, int nbase, const int* nbb, const int* blk0, const int64_t* tile0, int b, double* U,
                  double* Z, const unsigned char* nz, int* err) {
  if (b == 64)
    LIF_LAUNCH(k_potrf<64>, dim3(nbase), dim3(TileCfg<64>::THREADS), 0, c.stream, k, nbb, blk0, tile0, U, Z, nz,
               err);
  else
    LIF_LAUNCH(k_potrf<32>, dim3(nbase), dim3(TileCfg<32>::THREADS), 0, c.stream, k, nbb, blk0, tile0, U, Z, nz,
               err);
}

void launch_step(Ctx& c, int k, int band, int nbase, int max_nbb, const int* nbb, const int* blk0,
                 const int64_t* tile0, int b, double* U, double* Z, unsigned char* nz, int* err) {
  const int m = std::max(0, std::min(band, max_nbb - k - 1));
  const int nupd = m * (m + 1) / 2;
  const int nv = std::min(band, k);
  if (nupd + nv <= 0) return;
  const int ntask = nupd + nv;
  dim3 grid((unsigned)(ntask * nbase));
  if (b == 64)
    LIF_LAUNCH(k_step<64>, grid, dim3(TileCfg<64>::THREADS), 0, c.stream, k, band, nupd, ntask, nbase, nbb, blk0,
               tile0, U, Z, nz, err);
  else
    LIF_LAUNCH(k_step<32>, grid, dim3(TileCfg<32>::THREADS), 0, c.stream, k, band, nupd, ntask, nbase, nbb, blk0,
               tile0, U, Z, nz, err);
}

void launch_trinv(Ctx& c, int j0, int ncol, int band, int nbase, const int* nbb, const int64_t* tile0, int b,
                  const double* U, double* Z, const unsigned char* nz) {
  const int rows = j0 + ncol - 1;  // rows 0 .. j0 + ncol - 2 have a column of the range right of them
  if (ncol <= 0 || rows <= 0) return;
  dim3 grid(rows, nbase);
  if (b == 64)
    LIF_LAUNCH(k_trinv<64>, grid, dim3(TileCfg<64>::THREADS), 0, c.stream, j0, ncol, band, nbb, tile0, U, Z, nz);
  else
    LIF_LAUNCH(k_trinv<32>, grid, dim3(TileCfg<32>::THREADS), 0, c.stream, j0, ncol, band, nbb, tile0, U, Z, nz);
}

}  // namespace lif
