// Exclusive prefix sums of per-row counts (block-CSR row pointers, product
// offsets).  One workgroup of 1024 threads: each thread sums a contiguous
// chunk, the chunk totals are scanned in LDS, then each thread writes its
// chunk.  The arrays scanned here have one entry per block row (<= 2^15 on
// the supported sizes), so one workgroup is enough and the result is exact
// and deterministic.
#include "common.h"

namespace lif {

namespace {

constexpr int kScanThreads = 1024;

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_exclusive(const T* __restrict__ in,
                                                                  T* __restrict__ out, int count) {
  __shared__ T part[kScanThreads];
  const int t = threadIdx.x;
  const int chunk = (count + kScanThreads - 1) / kScanThreads;
  const int lo = min(count, t * chunk);
  const int hi = min(count, lo + chunk);
  T s = 0;
  for (int i = lo; i < hi; ++i) s += in[i];
  part[t] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan of the chunk totals
  for (int off = 1; off < kScanThreads; off <<= 1) {
    T v = (t >= off) ? part[t - off] : T(0);
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  T run = (t == 0) ? T(0) : part[t - 1];
  for (int i = lo; i < hi; ++i) {
    out[i] = run;
    run += in[i];
  }
  if (t == kScanThreads - 1) out[count] = part[kScanThreads - 1];
}

}  // namespace

void scan_exclusive_i32(Ctx& c, const int* in, int* out, int count) {
  hipLaunchKernelGGL(k_scan_exclusive<int>, dim3(1), dim3(kScanThreads), 0, c.stream, in, out, count);
  LIF_HIP(hipGetLastError());
}

void scan_exclusive_i64(Ctx& c, const int64_t* in, int64_t* out, int count) {
  hipLaunchKernelGGL(k_scan_exclusive<int64_t>, dim3(1), dim3(kScanThreads), 0, c.stream, in, out,
                     count);
  LIF_HIP(hipGetLastError());
}

}  // namespace lif
