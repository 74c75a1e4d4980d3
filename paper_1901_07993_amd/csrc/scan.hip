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

// both arrays in one launch: workgroup 0 scans the int32 array, workgroup 1
// the int64 array
__global__ __launch_bounds__(kScanThreads) void k_scan_pair(const int* __restrict__ in32, int* __restrict__ out32,
                                                            const int64_t* __restrict__ in64,
                                                            int64_t* __restrict__ out64, int count) {
  if (blockIdx.x == 0) {
    __shared__ int part[kScanThreads];
    const int t = threadIdx.x;
    const int chunk = (count + kScanThreads - 1) / kScanThreads;
    const int lo = min(count, t * chunk), hi = min(count, lo + chunk);
    int s = 0;
    for (int i = lo; i < hi; ++i) s += in32[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
      int v = (t >= off) ? part[t - off] : 0;
      __syncthreads();
      part[t] += v;
      __syncthreads();
    }
    int run = t ? part[t - 1] : 0;
    for (int i = lo; i < hi; ++i) {
      out32[i] = run;
      run += in32[i];
    }
    if (t == kScanThreads - 1) out32[count] = part[kScanThreads - 1];
  } else {
    __shared__ int64_t part64[kScanThreads];
    const int t = threadIdx.x;
    const int chunk = (count + kScanThreads - 1) / kScanThreads;
    const int lo = min(count, t * chunk), hi = min(count, lo + chunk);
    int64_t s = 0;
    for (int i = lo; i < hi; ++i) s += in64[i];
    part64[t] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
      int64_t v = (t >= off) ? part64[t - off] : 0;
      __syncthreads();
      part64[t] += v;
      __syncthreads();
    }
    int64_t run = t ? part64[t - 1] : 0;
    for (int i = lo; i < hi; ++i) {
      out64[i] = run;
      run += in64[i];
    }
    if (t == kScanThreads - 1) out64[count] = part64[kScanThreads - 1];
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
  __shared__ int64_t part[kScanThreads];
  const int t = threadIdx.x;
  const int chunk = (count + kScanThreads - 1) / kScanThreads;
  const int lo = min(count, t * chunk), hi = min(count, lo + chunk);
  int64_t total[2];
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    int64_t s = 0;
    for (int i = lo; i < hi; ++i) s += pass ? in64[i] : (int64_t)in32[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
      const int64_t v = (t >= off) ? part[t - off] : 0;
      __syncthreads();
      part[t] += v;
      __syncthreads();
    }
    int64_t run = t ? part[t - 1] : 0;
    for (int i = lo; i < hi; ++i) {
      if (pass) {
        out64[i] = run;
        run += in64[i];
      } else {
        out32[i] = (int)run;
        run += in32[i];
      }
    }
    total[pass] = part[kScanThreads - 1];
    __syncthreads();  // every thread has its total before the next pass reuses part
  }
  if (t == kScanThreads - 1) {
    out32[count] = (int)total[0];
    out64[count] = total[1];
  }
  if (t == 0) {
    sizes[0] = total[0];
    sizes[1] = total[1];
  }
  if (total[0] > cap32 || total[1] > cap64) {
    __syncthreads();  // the scan's own writes land first
    for (int i = t; i <= count; i += kScanThreads) {
      out32[i] = 0;
      out64[i] = 0;
    }
    if (t == 0) *overflow = 1;
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
  hipLaunchKernelGGL(k_scan_pair, dim3(2), dim3(kScanThreads), 0, c.stream, in32, out32, in64, out64, count);
  LIF_HIP(hipGetLastError());
}

void scan_exclusive_pair_capped(Ctx& c, const int* in32, int* out32, const int64_t* in64, int64_t* out64, int count,
                                int64_t cap32, int64_t cap64, int64_t* sizes, int* overflow) {
  hipLaunchKernelGGL(k_scan_pair_capped, dim3(1), dim3(kScanThreads), 0, c.stream, in32, out32, in64, out64, count,
                     cap32, cap64, sizes, overflow);
  LIF_HIP(hipGetLastError());
}

void scan_exclusive_i32(Ctx& c, const int* in, int* out, int count) {
  hipLaunchKernelGGL(k_scan_exclusive<int>, dim3(1), dim3(kScanThreads), 0, c.stream, in, out, count);
  LIF_HIP(hipGetLastError());
}

}  // namespace lif
