// Single-pass exclusive prefix sums over the rows of a launch, without a
// chain through the rows: the rows are taken in groups of 64.  Each
// workgroup takes its row from a ticket counter (so every lower row belongs
// to a workgroup that is already running or done) and publishes its row's
// value.  The workgroup of the last row of a group waits for the group's 64
// values and publishes their sum.  A row's exclusive prefix is then the sum
// of the group sums below its group plus the values of the rows below it in
// its group: two reads of at most 64 words per 64 groups, one word per lane.
// (A two-level form of the decoupled look-back of D. Merrill and M.
// Garland, "Single-pass Parallel Prefix Scan with Decoupled Look-back",
// 2016; with one-row tiles a chain of inclusive prefixes through the rows
// would serialize the whole grid.)
//
// A published word packs a nonzero tag, the launch's epoch (so words left
// by earlier launches read as not yet published) and a 48-bit value.  Every
// wait is bounded: after kLbSpin polls the prefix is reported unknown and
// the caller must flag its result as invalid.
#pragma once

#include <hip/hip_runtime.h>

namespace lif {

constexpr unsigned long long kLbTag = 1ull << 62;
constexpr unsigned long long kLbVal = (1ull << 48) - 1;
constexpr unsigned kLbEpochMask = 0x3fffu;
constexpr int kLbSpin = 1 << 16;

__device__ inline unsigned long long lb_word(unsigned epoch, unsigned long long v) {
  return kLbTag | ((unsigned long long)(epoch & kLbEpochMask) << 48) | (v & kLbVal);
}

__device__ inline void lb_store(unsigned long long* w, unsigned long long x) {
  __hip_atomic_store(w, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline unsigned long long lb_load(unsigned long long* w) {
  return __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// All lanes of one wave: waits until the words wa[lo + lane], wb[lo + lane]
// of the lanes below `count` are published, and returns their sums.  Lane
// `own` (if in range) takes the values (oa, ob) instead of reading them.
// False when the spin budget ran out.
__device__ inline bool lb_sum_window(unsigned long long* wa, unsigned long long* wb, int lo, int count,
                                     unsigned epoch, int own, unsigned long long oa, unsigned long long ob,
                                     unsigned long long* sa, unsigned long long* sb, int* spins) {
  const int lane = threadIdx.x & 63;
  const bool in = lane < count;
  for (;;) {
    unsigned long long xa = 0, xb = 0;
    bool valid = true;
    if (in && lane != own) {
      xa = lb_load(wa + lo + lane);
      xb = lb_load(wb + lo + lane);
      const unsigned long long ep = (unsigned long long)(epoch & kLbEpochMask);
      valid = (xa >> 62) == 1 && ((xa >> 48) & kLbEpochMask) == ep && (xb >> 62) == 1 &&
              ((xb >> 48) & kLbEpochMask) == ep;
    }
    if (__ballot(!valid) == 0ull) {
      const unsigned long long va = !in ? 0ull : (lane == own ? oa : (xa & kLbVal));
      const unsigned long long vb = !in ? 0ull : (lane == own ? ob : (xb & kLbVal));
      *sa += wave_sum_u64(va);
      *sb += wave_sum_u64(vb);
      return true;
    }
    if (++*spins > kLbSpin) return false;
    __builtin_amdgcn_s_sleep(1);
  }
}

// Row i's own values (a, b), published by one lane.
__device__ inline void lb_publish(unsigned long long* rows_a, unsigned long long* rows_b, int i, unsigned epoch,
                                  unsigned long long a, unsigned long long b) {
  lb_store(rows_a + i, lb_word(epoch, a));
  lb_store(rows_b + i, lb_word(epoch, b));
}

// Called by all lanes of one wave for row i of nb, after row i published
// its values (a, b) with lb_publish -- as early as possible, so that the
// rows above find them when they get here.  Publishes the group sums when
// row i closes its group and returns the exclusive prefixes of a and b over
// rows < i.  False if a lower row did not publish within the spin budget
// (the group sum is then published anyway, as zero, so that no other row
// waits on this one).
__device__ inline bool lb_resolve2(unsigned long long* rows_a, unsigned long long* rows_b,
                                   unsigned long long* grp_a, unsigned long long* grp_b, int i, int nb,
                                   unsigned epoch, unsigned long long a, unsigned long long b,
                                   unsigned long long* ea, unsigned long long* eb) {
  const int lane = threadIdx.x & 63;
  const int g = i >> 6, g0 = g << 6;
  int spins = 0;
  bool ok = true;
  if (i == min(nb, g0 + 64) - 1) {  // the group's last row publishes its sum
    unsigned long long ga = 0, gb = 0;
    ok = lb_sum_window(rows_a, rows_b, g0, i - g0 + 1, epoch, i - g0, a, b, &ga, &gb, &spins);
    if (lane == 0) {
      lb_store(grp_a + g, lb_word(epoch, ok ? ga : 0ull));
      lb_store(grp_b + g, lb_word(epoch, ok ? gb : 0ull));
    }
  }
  unsigned long long sa = 0, sb = 0;
  if (ok) ok = lb_sum_window(rows_a, rows_b, g0, i - g0, epoch, -1, 0, 0, &sa, &sb, &spins);
  for (int h = 0; ok && h < g; h += 64)
    ok = lb_sum_window(grp_a, grp_b, h, min(64, g - h), epoch, -1, 0, 0, &sa, &sb, &spins);
  *ea = sa;
  *eb = sb;
  return ok;
}

// Both steps at once (when there is nothing to do between them).
__device__ inline bool lb_exclusive2(unsigned long long* rows_a, unsigned long long* rows_b,
                                     unsigned long long* grp_a, unsigned long long* grp_b, int i, int nb,
                                     unsigned epoch, unsigned long long a, unsigned long long b,
                                     unsigned long long* ea, unsigned long long* eb) {
  if ((threadIdx.x & 63) == 0) lb_publish(rows_a, rows_b, i, epoch, a, b);
  return lb_resolve2(rows_a, rows_b, grp_a, grp_b, i, nb, epoch, a, b, ea, eb);
}

}  // namespace lif
