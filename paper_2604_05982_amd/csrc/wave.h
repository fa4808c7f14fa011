// wave.h -- wavefront-level primitives and memory-ordering helpers for gfx950.
//
// The paper publishes task IDs with a fence before the queue-size update and
// relies on one L2 shared by every SM as the coherence point (Sec. 2.3,
// Sec. 5.1.3).  On MI355X each XCD has its own L2, and an agent-scope
// release/acquire fence is a whole-L2 writeback/invalidate: measured on the
// device, such fences sustain only ~0.04-0.14 G wave-ops/s chip-wide while
// device-scope atomic loads, stores and relaxed RMWs sustain 1.4-9 G/s.
// So the runtime never uses agent-scope fences on its hot path.  Every datum
// one wavefront hands to another (frames, ring slots, depot chunks, candidate
// buffers, results) is written with a device-scope coherent store and read
// with a device-scope coherent load (co_st*/co_ld*: the "sc1" cache policy,
// performed at the device coherence point), and ordering between such
// accesses and the publishing RMW comes from drain(): the wavefront waits
// until every memory operation it issued has completed before issuing the
// next one.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.h"

#define GTAP_DEV __device__ __forceinline__

namespace gtap {

GTAP_DEV uint32_t lane_id() { return __lane_id(); }

GTAP_DEV uint64_t ballot(bool p) { return __ballot(p); }

// Number of set bits of m in lanes below this one.
GTAP_DEV uint32_t rank_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}

// Value of the first active lane (wave-uniform, lives in an SGPR).
GTAP_DEV uint32_t uniform(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
GTAP_DEV int32_t uniform(int32_t x) { return static_cast<int32_t>(__builtin_amdgcn_readfirstlane(static_cast<uint32_t>(x))); }
GTAP_DEV uint64_t uniform64(uint64_t x) {
  uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(x));
  uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(x >> 32));
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

// ---- cross-lane scans with DPP (VALU data-parallel primitives) ---------------
// Rows of 16 lanes: row_shr:n shifts within a row (lanes whose source lies
// outside the row read 0), row_bcast:15 / row_bcast:31 broadcast the last lane
// of row 0 (2) into rows 1,3 (2,3).  Must be called with every lane active.
enum DppCtrl : int {
  kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118,
  kRowBcast15 = 0x142, kRowBcast31 = 0x143
};

template <int CTRL, int ROWMASK>
GTAP_DEV uint32_t dpp_in(uint32_t x) {
  return static_cast<uint32_t>(
      __builtin_amdgcn_update_dpp(0, static_cast<int>(x), CTRL, ROWMASK, 0xF, true));
}
template <int CTRL, int ROWMASK>
GTAP_DEV uint64_t dpp_in64(uint64_t x) {
  const uint32_t lo = dpp_in<CTRL, ROWMASK>(static_cast<uint32_t>(x));
  const uint32_t hi = dpp_in<CTRL, ROWMASK>(static_cast<uint32_t>(x >> 32));
  return static_cast<uint64_t>(lo) | (static_cast<uint64_t>(hi) << 32);
}

// Inclusive prefix sum over the wave.
GTAP_DEV uint32_t wave_inclusive_sum(uint32_t x) {
  x += dpp_in<kRowShr1, 0xF>(x);
  x += dpp_in<kRowShr2, 0xF>(x);
  x += dpp_in<kRowShr4, 0xF>(x);
  x += dpp_in<kRowShr8, 0xF>(x);
  x += dpp_in<kRowBcast15, 0xA>(x);
  x += dpp_in<kRowBcast31, 0xC>(x);
  return x;
}
GTAP_DEV uint64_t wave_inclusive_sum64(uint64_t x) {
  x += dpp_in64<kRowShr1, 0xF>(x);
  x += dpp_in64<kRowShr2, 0xF>(x);
  x += dpp_in64<kRowShr4, 0xF>(x);
  x += dpp_in64<kRowShr8, 0xF>(x);
  x += dpp_in64<kRowBcast15, 0xA>(x);
  x += dpp_in64<kRowBcast31, 0xC>(x);
  return x;
}
// Inclusive prefix maximum (values >= 0).
GTAP_DEV uint32_t wave_inclusive_max(uint32_t x) {
  uint32_t y;
  y = dpp_in<kRowShr1, 0xF>(x); x = x > y ? x : y;
  y = dpp_in<kRowShr2, 0xF>(x); x = x > y ? x : y;
  y = dpp_in<kRowShr4, 0xF>(x); x = x > y ? x : y;
  y = dpp_in<kRowShr8, 0xF>(x); x = x > y ? x : y;
  y = dpp_in<kRowBcast15, 0xA>(x); x = x > y ? x : y;
  y = dpp_in<kRowBcast31, 0xC>(x); x = x > y ? x : y;
  return x;
}

// Value of the lane below / above; lane 0 / lane 63 receive `fill`.  Like
// every DPP helper here it must run with all 64 lanes active: call it
// unconditionally (a disabled source lane would read as `fill`).
GTAP_DEV uint32_t wave_from_below(uint32_t x, uint32_t fill) {
  return static_cast<uint32_t>(
      __builtin_amdgcn_update_dpp(static_cast<int>(fill), static_cast<int>(x), 0x138, 0xF, 0xF, false));
}
GTAP_DEV uint32_t wave_from_above(uint32_t x, uint32_t fill) {
  return static_cast<uint32_t>(
      __builtin_amdgcn_update_dpp(static_cast<int>(fill), static_cast<int>(x), 0x130, 0xF, 0xF, false));
}

// Lane k's 64-bit value x (k wave-uniform), as two 32-bit lane reads.
GTAP_DEV uint64_t readlane64(uint64_t x, int k) {
  const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(x)), k));
  const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(x >> 32)), k));
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Exclusive prefix sum over the 64 lanes; *total = sum over all lanes.
GTAP_DEV uint32_t wave_exclusive_scan(uint32_t x, uint32_t *total) {
  const uint32_t s = wave_inclusive_sum(x);
  *total = __builtin_amdgcn_readlane(s, 63);
  return s - x;
}

// ---- device-scope atomics (relaxed; ordering comes from drain()) ----------
template <typename T>
GTAP_DEV T ld_relaxed(T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
GTAP_DEV void st_relaxed(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
GTAP_DEV T fetch_add_relaxed(T *p, T v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
GTAP_DEV T fetch_or_relaxed(T *p, T v) {
  return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// CAS; on failure *expected receives the current value.
template <typename T>
GTAP_DEV bool cas_relaxed(T *p, T *expected, T desired) {
  return __hip_atomic_compare_exchange_strong(p, expected, desired, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- device-coherent data accesses -----------------------------------------
GTAP_DEV void co_st32(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
GTAP_DEV void co_st64(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
GTAP_DEV uint32_t co_ld32(const uint32_t *p) {
  return __hip_atomic_load(const_cast<uint32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
GTAP_DEV int32_t co_ld32i(const int32_t *p) {
  return __hip_atomic_load(const_cast<int32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
GTAP_DEV void co_st32i(int32_t *p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
GTAP_DEV uint64_t co_ld64(const uint64_t *p) {
  return __hip_atomic_load(const_cast<uint64_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- system-scope accesses (pinned host memory shared with the host) ------
GTAP_DEV uint64_t sys_ld64(const uint64_t *p) {
  return __hip_atomic_load(const_cast<uint64_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
GTAP_DEV int32_t sys_ld32i(const int32_t *p) {
  return __hip_atomic_load(const_cast<int32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
GTAP_DEV void sys_st64(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Wait until every memory operation this wavefront has issued is complete
// (stores and RMWs performed at their coherence point, loads returned).  The
// wavefront-scope fences keep the compiler from moving memory accesses across
// the wait.
GTAP_DEV void drain() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
}

// Orders LDS and global accesses between the lanes of one wavefront.
GTAP_DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Constant-rate device clock (rate: hipDeviceAttributeWallClockRate).
GTAP_DEV uint64_t wall_ticks() { return __builtin_amdgcn_s_memrealtime(); }

// Idle backoff: s_sleep k waits about 64*k cycles; k is an immediate.
GTAP_DEV void backoff_sleep(uint32_t n) {
  if (n < 2) __builtin_amdgcn_s_sleep(2);
  else if (n < 8) __builtin_amdgcn_s_sleep(8);
  else if (n < 32) __builtin_amdgcn_s_sleep(24);
  else __builtin_amdgcn_s_sleep(64);
}

// xorshift32 step (Marsaglia 2003); wave-uniform state.
GTAP_DEV uint32_t xorshift32(uint32_t &s) {
  s ^= s << 13;
  s ^= s >> 17;
  s ^= s << 5;
  return s;
}

}  // namespace gtap
