// fmm_lists.h -- the FMM pipeline of GTaP Sec. 6.4.1: the dual-tree traversal
// only builds interaction lists (well-separated cell pairs for M2L, leaf
// pairs for P2P) in fixed-capacity arrays appended with atomic adds; the lists
// are then sorted by target and evaluated by the data-parallel kernels of
// fmm_eval.h.  Two traversals build them:
// thread-mode tasks of the runtime (one cell pair per task, see tasks.h) and a
// level-synchronous worklist (ping-pong frontiers, one launch per frontier).
//
// MI355X choice: appends are aggregated per wavefront (one atomic per
// wavefront and list).
#pragma once
#include "fmm.h"
#include "wave.h"

namespace gtap {
namespace fmm {

// The cell-pair decision, the same in every traversal (the oracle's rule):
// 1 = accepted by the MAC (M2L), 2 = two leaves (P2P), 0 = split the wider
// cell (on equal levels the target unless it is a leaf; never a leaf), with
// split_a telling which.
GTAP_DEV uint32_t dtt_decide(const int32_t *A, const int32_t *B, int64_t ta, int64_t tb, bool &split_a) {
  split_a = false;
  if (mac_accept(A, B, ta, tb)) return 1;
  if (A[7] == 0 && B[7] == 0) return 2;
  bool s = A[0] < B[0] ? true : (A[0] > B[0] ? false : A[7] != 0);
  if (s && A[7] == 0) s = false;
  if (!s && B[7] == 0) s = true;
  split_a = s;
  return 0;
}

GTAP_DEV uint64_t readlane64(uint64_t v, int lane) {
  const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v)), lane));
  const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v >> 32)), lane));
  return static_cast<uint64_t>(lo) | (static_cast<uint64_t>(hi) << 32);
}

// Append `pair` to list `which` (0 = M2L, 1 = P2P) of each active lane's
// descriptor: one atomic add per wavefront and descriptor.  Entries past the
// capacity are counted but not stored.  Every lane of the wavefront calls it.
GTAP_DEV void list_append(FmmDesc *D, uint32_t which, bool act, uint64_t pair) {
  uint64_t m = ballot(act);
  while (m != 0ull) {
    const int leader = __ffsll(static_cast<long long>(m)) - 1;
    const uint64_t dl = readlane64(reinterpret_cast<uint64_t>(D), leader);
    const bool same = act && reinterpret_cast<uint64_t>(D) == dl;
    const uint64_t ms = ballot(same);
    uint64_t base = 0;
    if (static_cast<int>(lane_id()) == leader)
      base = fetch_add_relaxed(which ? &D->p2p_n : &D->m2l_n, static_cast<uint64_t>(__popcll(ms)));
    base = readlane64(base, leader);
    if (same) {
      const uint64_t idx = base + rank_below(ms);
      if (idx < (which ? D->p2p_cap : D->m2l_cap)) (which ? D->p2p_list : D->m2l_list)[idx] = pair;
    }
    m &= ~ms;
  }
}

// Chunked appends of a persistent wavefront (thread-mode traversal tasks): the
// wavefront reserves kListChunk slots with one atomic add and fills them over
// many iterations, so the two list counters see one atomic per 2,048 pairs
// instead of one per wavefront and iteration (hundreds of wavefronts adding to
// one word serialise).  Slots a wavefront leaves unused when it moves on hold
// the gap pair (ncells << 32), which sorts after every real target and is
// skipped by the evaluation.
constexpr uint32_t kListChunk = 2048;

struct ListChunks {
  FmmDesc *D;          // descriptor the chunks belong to (nullptr: none)
  uint64_t base[2];    // first slot of the current chunk, per list
  uint32_t used[2];    // slots of it filled
};

GTAP_DEV uint64_t gap_pair(const FmmDesc *D) { return static_cast<uint64_t>(D->ncells) << 32; }

// Fill the unused rest of both chunks with gaps (all lanes; wave-uniform state).
GTAP_DEV void chunks_close(ListChunks &C) {
  if (C.D == nullptr) return;
  for (uint32_t w = 0; w < 2; ++w) {
    const uint64_t cap = w ? C.D->p2p_cap : C.D->m2l_cap;
    uint64_t *list = w ? C.D->p2p_list : C.D->m2l_list;
    for (uint32_t i = C.used[w] + lane_id(); i < kListChunk; i += kWave) {
      const uint64_t at = C.base[w] + i;
      if (at < cap) list[at] = gap_pair(C.D);
    }
    C.used[w] = kListChunk;
  }
  C.D = nullptr;
}

// Append `pair` to list `which` for every active lane whose descriptor is the
// chunks' one (a wavefront's lanes almost always share it: a different one
// closes the chunks and takes over; lanes of a third go through list_append).
GTAP_DEV void chunks_append(ListChunks &C, FmmDesc *D, uint32_t which, bool act, uint64_t pair) {
  const uint64_t m = ballot(act);
  if (m == 0ull) return;
  const int leader = __ffsll(static_cast<long long>(m)) - 1;
  FmmDesc *dl = reinterpret_cast<FmmDesc *>(readlane64(reinterpret_cast<uint64_t>(D), leader));
  if (dl != C.D) {
    chunks_close(C);
    C.D = dl;
    C.used[0] = C.used[1] = kListChunk;  // no chunk reserved yet
  }
  const bool mine = act && D == dl;
  const uint64_t ms = ballot(mine);
  const uint32_t n = static_cast<uint32_t>(__popcll(ms));
  const uint32_t r = rank_below(ms);
  const uint64_t cap = which ? dl->p2p_cap : dl->m2l_cap;
  uint64_t *list = which ? dl->p2p_list : dl->m2l_list;
  // the part that fits in the current chunk, then a new chunk for the rest
  const uint32_t room = kListChunk - C.used[which];
  if (mine && r < room) {
    const uint64_t at = C.base[which] + C.used[which] + r;
    if (at < cap) list[at] = pair;
  }
  if (n > room) {
    uint64_t b = 0;
    if (lane_id() == 0) b = fetch_add_relaxed(which ? &dl->p2p_n : &dl->m2l_n, static_cast<uint64_t>(kListChunk));
    C.base[which] = readlane64(b, 0);
    C.used[which] = 0;
    if (mine && r >= room) {
      const uint64_t at = C.base[which] + (r - room);
      if (at < cap) list[at] = pair;
    }
    C.used[which] = n - room;
  } else {
    C.used[which] += n;
  }
  list_append(D, which, act && !mine, pair);
}

GTAP_DEV void load_cell(const int32_t *cell, uint32_t c, int32_t *C) {
  const int4 *p = reinterpret_cast<const int4 *>(cell + static_cast<size_t>(c) * kCellInts);
  const int4 u = p[0], v = p[1];
  C[0] = u.x; C[1] = u.y; C[2] = u.z; C[3] = u.w;
  C[4] = v.x; C[5] = v.y; C[6] = v.z; C[7] = v.w;
}

// ---- level-synchronous worklist traversal ------------------------------------
// One thread per pair of the frontier: accepted pairs and leaf pairs go to the
// lists, the child pairs of a split go to the next frontier.  Appends are
// aggregated over the 1,024-thread workgroup: one atomic add per workgroup
// and counter (the three counters are the hot words of this traversal).
// *nout keeps counting past cap_out.
constexpr uint32_t kFrontierThreads = 1024;

__global__ __launch_bounds__(kFrontierThreads) void k_dtt_frontier(FmmDesc *D, const uint64_t *fin, uint64_t nin,
                                                                   uint64_t *fout, uint64_t *nout, uint64_t cap_out) {
  constexpr uint32_t W = kFrontierThreads / kWave;
  __shared__ uint32_t wcnt[3][W];
  __shared__ uint64_t wbase[3][W];
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const uint32_t wv = threadIdx.x / kWave;
  const bool act = i < nin;
  uint64_t pair = 0;
  uint32_t dec = 3, k = 0, child0 = 0, a = 0, b = 0;
  bool split_a = false;
  if (act) {
    pair = fin[i];
    a = static_cast<uint32_t>(pair >> 32);
    b = static_cast<uint32_t>(pair);
    int32_t A[kCellInts], B[kCellInts];
    load_cell(D->cell, a, A);
    load_cell(D->cell, b, B);
    dec = dtt_decide(A, B, D->ta, D->tb, split_a);
    if (dec == 0) {
      k = static_cast<uint32_t>(split_a ? A[7] : B[7]);
      child0 = static_cast<uint32_t>(split_a ? A[6] : B[6]);
    }
  }
  // per-wavefront counts and offsets
  const uint64_t m1 = ballot(dec == 1), m2 = ballot(dec == 2);
  uint32_t ktot = 0;
  const uint32_t koff = wave_exclusive_scan(k, &ktot);
  if (lane_id() == 0) {
    wcnt[0][wv] = static_cast<uint32_t>(__popcll(m1));
    wcnt[1][wv] = static_cast<uint32_t>(__popcll(m2));
    wcnt[2][wv] = ktot;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const uint32_t c = threadIdx.x;
    uint32_t tot = 0;
    for (uint32_t w = 0; w < W; ++w) tot += wcnt[c][w];
    uint64_t base = 0;
    if (tot) base = fetch_add_relaxed(c == 0 ? &D->m2l_n : c == 1 ? &D->p2p_n : nout, static_cast<uint64_t>(tot));
    for (uint32_t w = 0; w < W; ++w) {
      wbase[c][w] = base;
      base += wcnt[c][w];
    }
  }
  __syncthreads();
  if (dec == 1) {
    const uint64_t at = wbase[0][wv] + rank_below(m1);
    if (at < D->m2l_cap) D->m2l_list[at] = pair;
  } else if (dec == 2) {
    const uint64_t at = wbase[1][wv] + rank_below(m2);
    if (at < D->p2p_cap) D->p2p_list[at] = pair;
  }
  const uint64_t base = wbase[2][wv] + koff;
  for (uint32_t j = 0; j < k; ++j) {
    const uint32_t c = child0 + j;
    if (base + j < cap_out)
      fout[base + j] = split_a ? ((static_cast<uint64_t>(c) << 32) | b) : ((static_cast<uint64_t>(a) << 32) | c);
  }
}

// ---- list evaluation ------------------------------------------------------------
// Segment [lo[a], hi[a]) of target a in a list sorted by target (both zeroed
// beforehand, so targets without pairs have empty segments; a = ncells, the
// gaps, gets a segment of its own that nothing reads).
__global__ void k_list_segments(const uint64_t *pairs, uint64_t n, uint64_t *lo, uint64_t *hi) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t a = static_cast<uint32_t>(pairs[i] >> 32);
  if (i == 0 || static_cast<uint32_t>(pairs[i - 1] >> 32) != a) lo[a] = i;
  if (i + 1 == n || static_cast<uint32_t>(pairs[i + 1] >> 32) != a) hi[a] = i + 1;
}

// Order-independent wrapping sum of pair hashes of a list (the oracle's check)
// and the number of real pairs (gaps, target == ncells, are skipped).
__global__ __launch_bounds__(256) void k_list_hash(const uint64_t *pairs, uint64_t n, uint32_t ncells, uint64_t *out,
                                                   uint64_t *count) {
  uint64_t h = 0, k = 0;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint32_t a = static_cast<uint32_t>(pairs[i] >> 32);
    if (a >= ncells) continue;
    h += pair_hash(a, static_cast<uint32_t>(pairs[i]));
    ++k;
  }
  h = readlane64(wave_inclusive_sum64(h), 63);
  k = readlane64(wave_inclusive_sum64(k), 63);
  if (lane_id() == 0 && h) fetch_add_relaxed(out, h);
  if (lane_id() == 0 && k) fetch_add_relaxed(count, k);
}

// 1 / sqrt(x) for x > 0: the hardware estimate refined by two Newton-Raphson
// steps y <- y (3 - x y^2) / 2 (each squares the relative error).
GTAP_DEV double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}

}  // namespace fmm
}  // namespace gtap
