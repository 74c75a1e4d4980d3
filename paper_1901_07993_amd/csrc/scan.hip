// Exclusive prefix sums of per-row counts (block-CSR row pointers, product
// offsets).  One workgroup of 1024 threads: each thread sums a contiguous
// chunk, the chunk totals are scanned (block_scan.h), then each thread
// writes its chunk.  The arrays scanned here have one entry per block row (<= 2^15 on
// the supported sizes), so one workgroup is enough and the result is exact
// and deterministic.
#include "block_scan.h"
#include "common.h"

namespace lif {

namespace {

constexpr int kScanThreads = 1024;

// Each thread sums a contiguous chunk of the input, the chunk totals are
// scanned, then each thread writes its chunk's prefix sums.
template <typename T, typename In>
__device__ void scan_chunks(const In* __restrict__ in, T* __restrict__ out, int count, T* sh, T* total) {
  const int t = threadIdx.x;
  const int chunk = (count + kScanThreads - 1) / kScanThreads;
  const int lo = min(count, t * chunk), hi = min(count, lo + chunk);
  T s = 0;
  for (int i = lo; i < hi; ++i) s += (T)in[i];
  T run = block_exclusive_scan<T, kScanThreads>(s, sh, total);
  for (int i = lo; i < hi; ++i) {
    out[i] = run;
    run += (T)in[i];
  }
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_exclusive(const T* __restrict__ in,
                                                                  T* __restrict__ out, int count) {
  __shared__ T sh[kScanThreads / 64];
  T total;
  scan_chunks<T, T>(in, out, count, sh, &total);
  if (threadIdx.x == 0) out[count] = total;
}

// both arrays in one launch: workgroup 0 scans the int32 array, workgroup 1
// the int64 array
__global__ __launch_bounds__(kScanThreads) void k_scan_pair(const int* __restrict__ in32, int* __restrict__ out32,
                                                            const int64_t* __restrict__ in64,
                                                            int64_t* __restrict__ out64, int count) {
  __shared__ int64_t sh[kScanThreads / 64];
  if (blockIdx.x == 0) {
    int total;
    scan_chunks<int, int>(in32, out32, count, reinterpret_cast<int*>(sh), &total);
    if (threadIdx.x == 0) out32[count] = total;
  } else {
    int64_t total;
    scan_chunks<int64_t, int64_t>(in64, out64, count, sh, &total);
    if (threadIdx.x == 0) out64[count] = total;
  }
}

// Both scans in one workgroup against capacities fixed before the counts
// were known.  When a total exceeds its capacity both row pointers are
// zeroed, so every later kernel sees a valid empty product, and the flag is
// raised for the host to redo the work with exact sizes.
__global__ __launch_bounds__(kScanThreads) void k_scan_pair_capped(const int* __restrict__ in32,
                                                                   int* __restrict__ out32,
                                                                   const int64_t* __restrict__ in64,
                                                                   int64_t* __restrict__ out64, int count,
                                                                   int64_t cap32, int64_t cap64,
                                                                   int64_t* __restrict__ sizes,
                                                                   int* __restrict__ overflow) {
  __shared__ int64_t sh[kScanThreads / 64];
  int64_t total32, total64;
  {
    int t32;
    scan_chunks<int, int>(in32, out32, count, reinterpret_cast<int*>(sh), &t32);
    total32 = t32;
  }
  __syncthreads();  // sh is reused
  scan_chunks<int64_t, int64_t>(in64, out64, count, sh, &total64);
  if (threadIdx.x == 0) {
    out32[count] = (int)total32;
    out64[count] = total64;
    sizes[0] = total32;
    sizes[1] = total64;
  }
  if (total32 > cap32 || total64 > cap64) {
    __syncthreads();  // the scan's own writes land first
    for (int i = threadIdx.x; i <= count; i += kScanThreads) {
      out32[i] = 0;
      out64[i] = 0;
    }
    if (threadIdx.x == 0) *overflow = 1;
  }
}

// Copies up to 32 small device values (<= 64 bytes each) into slots of 64
// bytes of a mapped host buffer; one lane per byte.
__global__ void k_gather_bytes(const void* const* __restrict__ src, const unsigned* __restrict__ bytes, int count,
                               unsigned char* __restrict__ dst) {
  const int i = blockIdx.x;
  if (i >= count) return;
  const unsigned char* s = static_cast<const unsigned char*>(src[i]);
  for (unsigned t = threadIdx.x; t < bytes[i]; t += blockDim.x) dst[64 * i + t] = s[t];
  __threadfence_system();
}

}  // namespace

void launch_gather_bytes(hipStream_t stream, const void* const* src, const unsigned* bytes, int count, void* dst) {
  hipLaunchKernelGGL(k_gather_bytes, dim3(count), dim3(64), 0, stream, src, bytes, count,
                     static_cast<unsigned char*>(dst));
  LIF_HIP(hipGetLastError());
}

void scan_exclusive_pair(Ctx& c, const int* in32, int* out32, const int64_t* in64, int64_t* out64, int count) {
  hipEvent_t t0 = c.timed_begin(2);  // part of the symbolic phase
  hipLaunchKernelGGL(k_scan_pair, dim3(2), dim3(kScanThreads), 0, c.stream, in32, out32, in64, out64, count);
  LIF_HIP(hipGetLastError());
  c.timed_end(t0, Ctx::Symbolic);
}

void scan_exclusive_pair_capped(Ctx& c, const int* in32, int* out32, const int64_t* in64, int64_t* out64, int count,
                                int64_t cap32, int64_t cap64, int64_t* sizes, int* overflow) {
  hipEvent_t t0 = c.timed_begin(2);  // part of the symbolic phase
  hipLaunchKernelGGL(k_scan_pair_capped, dim3(1), dim3(kScanThreads), 0, c.stream, in32, out32, in64, out64, count,
                     cap32, cap64, sizes, overflow);
  LIF_HIP(hipGetLastError());
  c.timed_end(t0, Ctx::Symbolic);
}

void scan_exclusive_i32(Ctx& c, const int* in, int* out, int count) {
  hipLaunchKernelGGL(k_scan_exclusive<int>, dim3(1), dim3(kScanThreads), 0, c.stream, in, out, count);
  LIF_HIP(hipGetLastError());
}

}  // namespace lif
