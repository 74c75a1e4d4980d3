// lif_multiply_noalloc: the block-sparse product of lif_multiply_add for
// callers that cannot allocate.  Its working memory is one file-scope device
// array per GPU; the product code runs unchanged on a pool that carves every
// buffer from that array and never calls hipMalloc / hipFree, with read-backs
// copied straight into host memory (no pinned staging).
#include <cmath>
#include <mutex>

#include "common.h"

namespace lif {
namespace {

constexpr size_t kScratchBytes = (size_t)LIF_NOALLOC_SCRATCH_BYTES;

// In host code `scratch` is a stand-in for the symbol, not a device address:
// only the address taken by hipGetSymbolAddress below is passed on.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
struct DeviceScratch {
  std::mutex mu;       // serializes the calls on this GPU
  void* ptr = nullptr; // this GPU's copy of `scratch`, once taken
};
DeviceScratch g_scratch[kMaxDevices];

// Device address of the current GPU's copy of `scratch`, taken once per
// device with that device current (the caller holds the device's lock).
void* scratch_address(DeviceScratch& d) {
  if (!d.ptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      throw Error(LIF_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    d.ptr = p;
  }
  return d.ptr;
}

void run(const lif_blocks* A, int32_t transA, const lif_blocks* B, int32_t transB, double alpha,
         const lif_blocks* D, double gamma, double tau, int32_t prec, hipStream_t stream, int64_t capacity,
         int64_t* nnzb, int32_t* brow, int32_t* bcol, double* vals, int64_t* products, void* base) {
  LIF_REQUIRE(nnzb != nullptr, LIF_ERR_INVALID, "nnzb is null");
  LIF_REQUIRE(std::isfinite(tau) && tau >= 0.0, LIF_ERR_INVALID, "tau must be finite and >= 0");
  LIF_REQUIRE(std::isfinite(alpha) && std::isfinite(gamma), LIF_ERR_INVALID, "alpha and gamma must be finite");
  LIF_REQUIRE(prec == LIF_FP64 || prec == LIF_MIXED_FP32 || prec == LIF_MIXED_BF16, LIF_ERR_INVALID,
              "prec is invalid");
  LIF_REQUIRE((transA & ~(1 | LIF_PRODUCT_UPPER)) == 0 && (transB & ~1) == 0, LIF_ERR_INVALID,
              "transA / transB: unknown flags");
  LIF_REQUIRE(capacity >= 0, LIF_ERR_INVALID, "capacity must be >= 0");
  validate_blocks(A, false, "A");
  validate_blocks(B, false, "B");
  if (D) validate_blocks(D, false, "D");
  LIF_REQUIRE(A->on_device && B->on_device && (!D || D->on_device), LIF_ERR_INVALID,
              "lif_multiply_noalloc takes device block lists only (on_device = 1)");
  LIF_REQUIRE(A->n == B->n && A->b == B->b && (!D || (D->n == A->n && D->b == A->b)), LIF_ERR_INVALID,
              "A, B and D must have the same n and b");
  // the pool is declared first so that every buffer (context, matrices) is
  // handed back to it before it goes
  Pool pool(base, kScratchBytes);
  Ctx c;
  c.stream = stream;
  c.pool = &pool;
  c.no_host_alloc = true;
  c.b = A->b;
  c.n = A->n;
  c.nb = (int)((A->n + A->b - 1) / A->b);
  try {
    Bsr a = bsr_view_blocks(c, *A);
    Bsr b = bsr_view_blocks(c, *B);
    Bsr d;
    if (D) d = bsr_view_blocks(c, *D);
    Bsr C = spgemm(c, a, (transA & 1) != 0, b, (transB & 1) != 0, tau, prec, alpha, D ? &d : nullptr,
                   D ? gamma : 0.0, false, false, (transA & LIF_PRODUCT_UPPER) != 0);
    const int64_t have = exact_nnzb(c, C);
    if (products) *products = c.stats.products;
    if (have > capacity) {
      *nnzb = have;
      throw Error(LIF_ERR_INVALID, "output capacity " + std::to_string(capacity) + " < " + std::to_string(have) +
                                       " blocks");
    }
    LIF_REQUIRE(have == 0 || (brow && bcol && vals), LIF_ERR_INVALID, "null output array");
    bsr_to_blocks(c, C, brow, bcol, vals, true);
    *nnzb = have;
    c.sync();
  } catch (const Error& e) {
    // nothing queued may outlive the call: the next one reuses the array
    (void)hipStreamSynchronize(stream);
    if (e.status == LIF_ERR_OUT_OF_MEMORY)
      throw Error(LIF_ERR_OUT_OF_MEMORY, std::string("the product does not fit the ") +
                                             std::to_string(kScratchBytes >> 20) +
                                             " MiB scratch array of lif_multiply_noalloc (" + e.what() + ")");
    throw;
  }
}

}  // namespace
}  // namespace lif

extern "C" lif_status lif_multiply_noalloc(const lif_blocks* A, int32_t transA, const lif_blocks* B,
                                           int32_t transB, double alpha, const lif_blocks* D, double gamma,
                                           double tau, int32_t prec, void* stream, int64_t capacity, int64_t* nnzb,
                                           int32_t* brow, int32_t* bcol, double* vals, int64_t* products) {
  using namespace lif;
  try {
    int dev = -1;
    LIF_HIP(hipGetDevice(&dev));
    LIF_REQUIRE(dev >= 0 && dev < kMaxDevices, LIF_ERR_INVALID, "device ordinal out of range");
    DeviceScratch& d = g_scratch[dev];
    std::lock_guard<std::mutex> lock(d.mu);
    void* base = scratch_address(d);
    run(A, transA, B, transB, alpha, D, gamma, tau, prec, static_cast<hipStream_t>(stream), capacity, nnzb, brow,
        bcol, vals, products, base);
    return LIF_OK;
  } catch (const Error& e) {
    set_thread_error(e.what());
    return e.status;
  } catch (const std::bad_alloc&) {
    set_thread_error("host allocation failed");
    return LIF_ERR_OUT_OF_MEMORY;
  } catch (const std::exception& e) {
    set_thread_error(e.what());
    return LIF_ERR_HIP;
  }
}
