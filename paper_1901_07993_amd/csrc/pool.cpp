// Device memory pool and execution context.
#include "common.h"

namespace lif {

size_t Pool::round(size_t bytes) {
  // 256-byte granularity below 1 MiB, 1 MiB above: keeps reuse high for the
  // repeated, similarly sized buffers of the refinement loop.
  if (bytes < (1u << 20)) return (bytes + 255) & ~size_t(255);
  return (bytes + (1u << 20) - 1) & ~size_t((1u << 20) - 1);
}

void* Pool::alloc(size_t bytes) {
  size_t r = round(bytes);
  // smallest cached buffer that fits and wastes at most a quarter
  auto it = cache_.lower_bound(r);
  if (it != cache_.end() && it->first <= r + r / 4) {
    void* p = it->second;
    r = it->first;
    cache_.erase(it);
    live_[p] = r;
    in_use_ += r;
    if (in_use_ > peak_) peak_ = in_use_;
    return p;
  }
  if (cap_ && reserved_ + r > cap_) trim();
  if (cap_ && reserved_ + r > cap_)
    throw Error(LIF_ERR_OUT_OF_MEMORY, "device memory cap exceeded: need " + std::to_string(r) +
                                           " more bytes with " + std::to_string(reserved_) +
                                           " held, cap " + std::to_string(cap_));
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, r);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    trim();
    e = hipMalloc(&p, r);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(LIF_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(r) + " bytes failed");
    }
  }
  reserved_ += r;
  live_[p] = r;
  in_use_ += r;
  if (in_use_ > peak_) peak_ = in_use_;
  return p;
}

void Pool::free(void* p) {
  auto it = live_.find(p);
  if (it == live_.end()) return;
  if (defer_) {
    deferred_.push_back(p);
    return;
  }
  in_use_ -= it->second;
  cache_.emplace(it->second, p);
  live_.erase(it);
}

void Pool::release_deferred() {
  const bool keep = defer_;
  defer_ = false;
  for (void* p : deferred_) free(p);
  deferred_.clear();
  defer_ = keep;
}

void Pool::trim() {
  if (cache_.empty()) return;
  // memory in the cache may still be read by queued kernels of the stream
  // that freed it; wait for the device before giving it back
  (void)hipDeviceSynchronize();
  for (auto& kv : cache_) {
    (void)hipFree(kv.second);
    reserved_ -= kv.first;
  }
  cache_.clear();
}

void Pool::release_all() {
  (void)hipDeviceSynchronize();
  for (auto& kv : cache_) (void)hipFree(kv.second);
  for (auto& kv : live_) (void)hipFree(kv.first);
  cache_.clear();
  live_.clear();
  reserved_ = in_use_ = 0;
}

hipEvent_t Ctx::take_event() {
  if (!ev_free.empty()) {
    hipEvent_t e = ev_free.back();
    ev_free.pop_back();
    return e;
  }
  hipEvent_t e;
  LIF_HIP(hipEventCreate(&e));
  return e;
}

void Ctx::flush_timing() {
  if (ev_pending.empty()) return;
  LIF_HIP(hipStreamSynchronize(stream));
  for (auto& pr : ev_pending) {
    float ms = 0.f;
    LIF_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
    stats.gemm_ms += ms;
    ev_free.push_back(pr.first);
    ev_free.push_back(pr.second);
  }
  ev_pending.clear();
}

void launch_gather_bytes(hipStream_t stream, const void* const* src, const unsigned* bytes, int count, void* dst);

void Ctx::d2h(void* dst, const void* src, size_t bytes) {
  if (bytes <= 64) {
    d2h_batch({{dst, src, bytes}});
    return;
  }
  if (bytes > pinned_bytes) {
    if (pinned) (void)hipHostFree(pinned);
    pinned = nullptr;
    size_t want = bytes < 4096 ? 4096 : bytes;
    LIF_HIP(hipHostMalloc(&pinned, want, hipHostMallocDefault));
    pinned_bytes = want;
  }
  LIF_HIP(hipMemcpyAsync(pinned, src, bytes, hipMemcpyDeviceToHost, stream));
  LIF_HIP(hipStreamSynchronize(stream));
  std::memcpy(dst, pinned, bytes);
}

// Small reads: one kernel copies every requested value into a mapped pinned
// buffer (the GPU writes host memory directly), then one synchronization.
void Ctx::d2h_batch(const std::vector<Read>& reads) {
  const int n = (int)reads.size();
  LIF_REQUIRE(n <= 32, LIF_ERR_INVALID, "too many values in one read-back");
  if (!readback) {
    LIF_HIP(hipHostMalloc(&readback, 64 * 32 + 32 * (sizeof(void*) + sizeof(unsigned)), hipHostMallocMapped));
  }
  char* base = static_cast<char*>(readback);
  const void** srcs = reinterpret_cast<const void**>(base + 64 * 32);
  unsigned* lens = reinterpret_cast<unsigned*>(base + 64 * 32 + 32 * sizeof(void*));
  // the previous read-back has completed (it synchronized), so the argument
  // area may be rewritten
  for (int i = 0; i < n; ++i) {
    LIF_REQUIRE(reads[i].bytes <= 64, LIF_ERR_INVALID, "read-back value larger than 64 bytes");
    srcs[i] = reads[i].src;
    lens[i] = (unsigned)reads[i].bytes;
  }
  void* dev_args = nullptr;
  LIF_HIP(hipHostGetDevicePointer(&dev_args, readback, 0));
  char* dbase = static_cast<char*>(dev_args);
  launch_gather_bytes(stream, reinterpret_cast<const void* const*>(dbase + 64 * 32),
                      reinterpret_cast<const unsigned*>(dbase + 64 * 32 + 32 * sizeof(void*)), n, dbase);
  LIF_HIP(hipStreamSynchronize(stream));
  for (int i = 0; i < n; ++i) std::memcpy(reads[i].dst, base + 64 * i, reads[i].bytes);
}

hipStream_t Ctx::side_stream() {
  if (!side) LIF_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
  return side;
}

Ctx::Lookback& Ctx::lookback_for(int rows) {
  Lookback& lb = lookback[stream];
  if (!lb_fail.get()) {
    lb_fail = DBuf<int>(pool, 1);
    LIF_HIP(hipMemsetAsync(lb_fail.get(), 0, sizeof(int), stream));
  }
  if (lb.rows < rows) {
    // zeroed once: no word reads as published
    const size_t words = 2 * ((size_t)rows + Lookback::groups(rows));
    lb.words = DBuf<unsigned long long>(pool, words);
    LIF_HIP(hipMemsetAsync(lb.words.get(), 0, words * sizeof(unsigned long long), stream));
    lb.rows = rows;
  }
  return lb;
}

Ctx::LbWords Ctx::lookback_words(int rows) {
  Lookback& lb = lookback_for(rows);
  LbWords w;
  w.ra = lb.words.get();
  w.rb = w.ra + lb.rows;
  w.ga = w.rb + lb.rows;
  w.gb = w.ga + Lookback::groups(lb.rows);
  w.epoch = lb.next_epoch();
  w.fail = lb_fail.get();
  return w;
}

hipEvent_t Ctx::order_event(size_t i) {
  while (order_events.size() <= i) {
    hipEvent_t e = nullptr;
    LIF_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    order_events.push_back(e);
  }
  return order_events[i];
}

void Ctx::stream_after(hipStream_t waiter, hipStream_t signaler) {
  // a ring of events, far larger than the number of waits in flight between
  // two synchronizations of the host with the device
  if (ring_events.size() < 64) {
    hipEvent_t e = nullptr;
    LIF_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ring_events.push_back(e);
  }
  hipEvent_t e = ring_events[next_order % ring_events.size()];
  ++next_order;
  LIF_HIP(hipEventRecord(e, signaler));
  LIF_HIP(hipStreamWaitEvent(waiter, e, 0));
}

Ctx::~Ctx() {
  if (side) {
    (void)hipStreamSynchronize(side);
    (void)hipStreamDestroy(side);
  }
  for (auto e : order_events) (void)hipEventDestroy(e);
  for (auto e : ring_events) (void)hipEventDestroy(e);
  for (auto& pr : ev_pending) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  for (auto e : ev_free) (void)hipEventDestroy(e);
  if (pinned) (void)hipHostFree(pinned);
  if (readback) (void)hipHostFree(readback);
}

}  // namespace lif
