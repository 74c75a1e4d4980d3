// Device memory pool and execution context.
#include <cstdlib>

#include "common.h"

namespace lif {

size_t Pool::round(size_t bytes) {
  return (bytes + 255) & ~size_t(255);  // every buffer 256-byte aligned
}

Pool::Pool(void* base, size_t bytes) : cap_(bytes), fixed_(true) {
  char* b = static_cast<char*>(base);
  const size_t usable = bytes & ~size_t(255);
  segs_[b] = {usable, 0};
  pieces_[b] = Piece{usable, true, b};
  free_[0].insert({usable, b});
  reserved_ = reserved_cls_[0] = usable;
}

// A new segment for at least `need` bytes of class cls.  Small class: at
// least 64 MiB and half of what that class holds (up to 1 GiB).  Large class:
// at least 1 GiB, so that neighbouring large buffers can share one.
bool Pool::grow(size_t need, int cls) {
  if (fixed_) return false;
  constexpr size_t kGrain = size_t(2) << 20;
  size_t want = cls == 0 ? std::max(need, std::min(size_t(1) << 30,
                                                   std::max(size_t(64) << 20, (size_t)(reserved_cls_[0] / 2))))
                         : std::max(need, size_t(1) << 30);
  want = (want + kGrain - 1) & ~(kGrain - 1);
  if (cap_ && reserved_ + want > cap_) want = std::max(need, (size_t)(cap_ > reserved_ ? cap_ - reserved_ : 0));
  if (cap_ && reserved_ + want > cap_) return false;
  void* p = nullptr;
  if (hipMalloc(&p, want) != hipSuccess) {
    (void)hipGetLastError();
    if (want == need) return false;
    want = need;
    if (hipMalloc(&p, want) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
  }
  char* base = static_cast<char*>(p);
  segs_[base] = {want, cls};
  pieces_[base] = Piece{want, true, base};
  free_[cls].insert({want, base});
  reserved_ += want;
  reserved_cls_[cls] += want;
  ++seg_allocs_;
  return true;
}

// Marks the free piece `it` used for r bytes, splitting off the rest.
void Pool::take(std::map<char*, Piece>::iterator it, size_t r) {
  char* p = it->first;
  Piece& pc = it->second;
  const int cls = segs_[pc.seg].second;
  free_[cls].erase({pc.size, p});
  if (pc.size > r) {
    pieces_[p + r] = Piece{pc.size - r, true, pc.seg};
    free_[cls].insert({pc.size - r, p + r});
    pc.size = r;
  }
  pc.free = false;
  in_use_ += r;
  if (in_use_ > peak_) peak_ = in_use_;
}

void* Pool::alloc(size_t bytes) {
  const size_t r = round(bytes);
  const int cls = size_class(r);
  for (int attempt = 0; attempt < 3; ++attempt) {
    auto f = free_[cls].lower_bound({r, nullptr});  // best fit: the smallest free piece that fits
    if (f != free_[cls].end()) {
      auto it = pieces_.find(f->second);
      take(it, r);
      return it->first;
    }
    if (attempt == 0 && grow(r, cls)) continue;
    if (attempt == 1) {
      trim();  // give back whole unused segments, then try once more
      if (grow(r, cls)) continue;
    }
  }
  throw Error(LIF_ERR_OUT_OF_MEMORY, "device memory: cannot allocate " + std::to_string(r) + " bytes with " +
                                         std::to_string(reserved_) + " held (" + std::to_string(in_use_) +
                                         " in use)" + (cap_ ? ", cap " + std::to_string(cap_) : std::string()));
}

void Pool::free(void* ptr) {
  auto it = pieces_.find(static_cast<char*>(ptr));
  if (it == pieces_.end() || it->second.free) return;
  if (defer_) {
    deferred_.push_back(ptr);
    return;
  }
  const int cls = segs_[it->second.seg].second;
  in_use_ -= it->second.size;
  it->second.free = true;
  // merge with the free neighbours inside the same segment
  auto next = std::next(it);
  if (next != pieces_.end() && next->second.free && next->second.seg == it->second.seg) {
    free_[cls].erase({next->second.size, next->first});
    it->second.size += next->second.size;
    pieces_.erase(next);
  }
  if (it != pieces_.begin()) {
    auto prev = std::prev(it);
    if (prev->second.free && prev->second.seg == it->second.seg) {
      free_[cls].erase({prev->second.size, prev->first});
      prev->second.size += it->second.size;
      pieces_.erase(it);
      it = prev;
    }
  }
  free_[cls].insert({it->second.size, it->first});
}

bool Pool::shrink(void* ptr, size_t bytes) {
  auto it = pieces_.find(static_cast<char*>(ptr));
  if (it == pieces_.end() || it->second.free || defer_) return false;
  const size_t r = round(bytes);
  Piece& pc = it->second;
  if (r == 0 || r >= pc.size) return false;
  const int cls = segs_[pc.seg].second;
  char* tail = it->first + r;
  size_t tsize = pc.size - r;
  in_use_ -= tsize;
  pc.size = r;
  auto next = std::next(it);
  if (next != pieces_.end() && next->second.free && next->second.seg == pc.seg) {
    free_[cls].erase({next->second.size, next->first});
    tsize += next->second.size;
    pieces_.erase(next);
  }
  pieces_[tail] = Piece{tsize, true, pc.seg};
  free_[cls].insert({tsize, tail});
  return true;
}

void Pool::release_deferred() {
  const bool keep = defer_;
  defer_ = false;
  for (void* p : deferred_) free(p);
  deferred_.clear();
  defer_ = keep;
}

void Pool::trim() {
  if (fixed_) return;
  // a free segment may still be read by queued kernels of the stream that
  // freed its last buffer; wait for the device before giving it back
  bool synced = false;
  for (auto s = segs_.begin(); s != segs_.end();) {
    auto it = pieces_.find(s->first);
    if (it != pieces_.end() && it->second.free && it->second.size == s->second.first) {
      if (!synced) {
        (void)hipDeviceSynchronize();
        synced = true;
      }
      free_[s->second.second].erase({it->second.size, it->first});
      pieces_.erase(it);
      (void)hipFree(s->first);
      reserved_ -= s->second.first;
      reserved_cls_[s->second.second] -= s->second.first;
      s = segs_.erase(s);
    } else {
      ++s;
    }
  }
}

void Pool::release_all() {
  if (!fixed_) {
    (void)hipDeviceSynchronize();
    for (auto& kv : segs_) (void)hipFree(kv.first);
  }
  segs_.clear();
  pieces_.clear();
  free_[0].clear();
  free_[1].clear();
  deferred_.clear();
  reserved_ = in_use_ = 0;
  reserved_cls_[0] = reserved_cls_[1] = 0;
}

bool verbose() {
  static const bool on = std::getenv("LIF_VERBOSE") != nullptr;
  return on;
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

hipEvent_t Ctx::timed_begin(int level) {
  if (timing_level < level) return nullptr;
  hipEvent_t e = take_event();
  LIF_HIP(hipEventRecord(e, stream));
  return e;
}

void Ctx::timed_end(hipEvent_t e0, Timed what) {
  if (!e0) return;
  hipEvent_t e1 = take_event();
  LIF_HIP(hipEventRecord(e1, stream));
  ev_pending.emplace_back(e0, e1);
  ev_lowp.push_back(LIF_FP64);
  ev_cat.push_back((char)what);
  if (what == Leaf) ++stats.leaf_launches;
  if (what == Symbolic) ++stats.sym_launches;
}

void Ctx::flush_timing() {
  if (ev_pending.empty()) return;
  LIF_HIP(hipStreamSynchronize(stream));
  if (side) LIF_HIP(hipStreamSynchronize(side));  // events of the second stream as well
  for (size_t i = 0; i < ev_pending.size(); ++i) {
    auto& pr = ev_pending[i];
    float ms = 0.f;
    LIF_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
    const int cat = i < ev_cat.size() ? ev_cat[i] : Gemm;
    if (cat == Leaf) {
      stats.leaf_ms += ms;
    } else if (cat == Symbolic) {
      stats.sym_ms += ms;
    } else {
      stats.gemm_ms += ms;
      const int p = i < ev_lowp.size() ? ev_lowp[i] : LIF_FP64;
      if (p != LIF_FP64) stats.gemm_ms_lowp += ms;
      if (p == LIF_MIXED_FP32) stats.gemm_ms_f32 += ms;
    }
    ev_free.push_back(pr.first);
    ev_free.push_back(pr.second);
  }
  ev_pending.clear();
  ev_lowp.clear();
  ev_cat.clear();
}

void launch_gather_bytes(hipStream_t stream, const void* const* src, const unsigned* bytes, int count, void* dst);

void Ctx::d2h(void* dst, const void* src, size_t bytes) {
  if (no_host_alloc) {
    LIF_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, stream));
    LIF_HIP(hipStreamSynchronize(stream));
    return;
  }
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
  if (no_host_alloc) {
    for (const Read& r : reads) LIF_HIP(hipMemcpyAsync(r.dst, r.src, r.bytes, hipMemcpyDeviceToHost, stream));
    LIF_HIP(hipStreamSynchronize(stream));
    return;
  }
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

uint64_t Ctx::device_bytes() {
  if (!device_total) {
    size_t free_b = 0, total_b = 0;
    LIF_HIP(hipMemGetInfo(&free_b, &total_b));
    device_total = total_b;
  }
  return pool->cap() ? std::min<uint64_t>(pool->cap(), device_total) : device_total;
}

hipStream_t Ctx::side_stream() {
  if (!side) LIF_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
  return side;
}

Ctx::Lookback& Ctx::lookback_for(int rows) {
  Lookback& lb = lookback[stream];
  if (!lb_fail.get()) {
    lb_fail = DBuf<int>(pool, 1);
    if (no_host_alloc)
      launch_fill_i32(*this, lb_fail.get(), 0, 1);
    else
      LIF_HIP(hipMemsetAsync(lb_fail.get(), 0, sizeof(int), stream));
  }
  if (lb.rows < rows) {
    // zeroed once: no word reads as published
    const size_t words = 2 * ((size_t)rows + Lookback::groups(rows));
    lb.words = DBuf<unsigned long long>(pool, words);
    if (no_host_alloc)
      launch_fill_i32(*this, reinterpret_cast<int*>(lb.words.get()), 0, (int64_t)(2 * words));
    else
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
