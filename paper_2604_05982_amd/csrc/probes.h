// probes.h -- platform probes behind the runtime's design choices.
//
// atomic_probe_kernel measures the device-scope RMW rate the scheduler's
// roofline is priced against: every lane issues `iters` relaxed agent-scope
// 64-bit fetch-adds (with return, like the join-word updates) either on a
// word of its own (distinct 64-byte lines, like join words of different
// frames), on one word per wavefront issued by lane 0 (like a deque count),
// or on one word for the whole grid issued by lane 0 of every wavefront
// (fully contended).
//
// The litmus kernels check, between workgroups placed on different XCDs, the
// two orderings the runtime's hand-offs rely on when they use device-coherent
// relaxed accesses ordered by drain() instead of release/acquire fences:
//   message passing  writer: data = k; [drain]; flag = k      (k = 1, 2, ...)
//                    reader: f = flag; [drain]; d = data     -> d >= f
//   store buffering  A: x = r; [drain]; a_r = y
//                    B: y = r; [drain]; b_r = x              -> not (a_r < r and b_r < r)
// Every lane runs its own instance on its own 128-byte lines.  The loops run a
// fixed number of iterations with no waits, so every wavefront ends.
#pragma once
#include "wave.h"

namespace gtap {
namespace probe {

constexpr uint32_t kLineWords = 32;  // 128-byte lines of u32

__global__ void atomic_probe_kernel(uint64_t *words, uint32_t mode, uint32_t iters, uint64_t *sink) {
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t wave = gid / kWave;
  uint64_t *w = mode == 0 ? words + static_cast<size_t>(gid) * 8 : (mode == 1 ? words + static_cast<size_t>(wave) * 16 : words);
  const bool active = mode == 0 || lane_id() == 0;
  uint64_t acc = 0;
  if (active) {
    for (uint32_t i = 0; i < iters; ++i) acc += fetch_add_relaxed(w, static_cast<uint64_t>(1));
  }
  if (acc == 0x9E3779B97F4A7C15ull) sink[0] = acc;  // keeps the returned values live
}

// Hardware XCC (XCD) id of the executing wavefront: HW_REG_XCC_ID, bits [3:0].
GTAP_DEV uint32_t xcc_id() { return static_cast<uint32_t>(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20)); }

// Message passing.  Workgroup 2p writes, 2p+1 reads; lane l of pair p uses
// line pair (p * 64 + l).  out[pair * 64 + l] = {stale, observations of a
// flag strictly between 0 and rounds}.
template <bool kOrdered>
__global__ void litmus_mp_kernel(uint32_t *cells, uint32_t rounds, uint32_t reads, uint32_t *stale_out,
                                 uint32_t *mid_out, uint32_t *xcc) {
  const uint32_t pair = blockIdx.x >> 1, role = blockIdx.x & 1, ln = lane_id();
  const size_t inst = static_cast<size_t>(pair) * kWave + ln;
  uint32_t *data = cells + inst * 2 * kLineWords;
  uint32_t *flag = data + kLineWords;
  if (ln == 0) xcc[blockIdx.x] = xcc_id();
  if (role == 0) {
    for (uint32_t k = 1; k <= rounds; ++k) {
      co_st32(data, k);
      if (kOrdered) drain();
      co_st32(flag, k);
    }
  } else {
    uint32_t stale = 0, mid = 0;
    for (uint32_t r = 0; r < reads; ++r) {
      const uint32_t f = co_ld32(flag);
      if (kOrdered) drain();
      const uint32_t d = co_ld32(data);
      stale += d < f ? 1u : 0u;
      mid += (f > 0 && f < rounds) ? 1u : 0u;
    }
    stale_out[inst] = stale;
    mid_out[inst] = mid;
  }
}

// Store buffering.  Workgroup 2p is A, 2p+1 is B; obs[(inst * 2 + role) *
// rounds + r - 1] = the value the round-r load saw.
template <bool kOrdered>
__global__ void litmus_sb_kernel(uint32_t *cells, uint32_t rounds, uint32_t *obs, uint32_t *xcc) {
  const uint32_t pair = blockIdx.x >> 1, role = blockIdx.x & 1, ln = lane_id();
  const size_t inst = static_cast<size_t>(pair) * kWave + ln;
  uint32_t *x = cells + inst * 2 * kLineWords;
  uint32_t *y = x + kLineWords;
  uint32_t *mine = role == 0 ? x : y;
  const uint32_t *other = role == 0 ? y : x;
  uint32_t *o = obs + (inst * 2 + role) * rounds;
  if (ln == 0) xcc[blockIdx.x] = xcc_id();
  for (uint32_t r = 1; r <= rounds; ++r) {
    co_st32(mine, r);
    if (kOrdered) drain();
    o[r - 1] = co_ld32(other);
  }
}

// Outcome counts of the store-buffering rounds: [0] both loads saw the new
// value, [1] only A's, [2] only B's, [3] neither (forbidden if ordered).
__global__ void litmus_sb_count_kernel(const uint32_t *obs, uint32_t rounds, uint32_t instances,
                                       unsigned long long *counts) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= static_cast<size_t>(instances) * rounds) return;
  const size_t inst = i / rounds;
  const uint32_t r = static_cast<uint32_t>(i % rounds) + 1;
  const bool a_new = obs[(inst * 2 + 0) * rounds + r - 1] >= r;
  const bool b_new = obs[(inst * 2 + 1) * rounds + r - 1] >= r;
  const uint32_t k = a_new && b_new ? 0u : (a_new ? 1u : (b_new ? 2u : 3u));
  atomicAdd(counts + k, 1ull);
}

}  // namespace probe
}  // namespace gtap
