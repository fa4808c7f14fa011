// sched_thread.h -- persistent thread-mode scheduler for gfx950.
//
// Each 64-lane wavefront is one scheduler (GTaP Sec. 5.1.1, Algorithm 1,
// with a warp of 32 replaced by a wavefront of 64):
//   loop: top up the lanes [cnt,64) by a batched pop from the own deque, then
//         by a batched steal from a random victim; run one task per lane;
//         retain up to 64 of the task IDs made runnable in this iteration
//         (resumed parents first, then new children) and publish the rest
//         with one batched push; exit once every job's root has completed.
// Deques follow Sec. 5.1.3: a ring of task IDs with `head` (steal end) and
// `count` (unclaimed entries) in global memory, the owner-only `tail` in LDS,
// a lock per deque for thieves; every claim is a CAS on `count`; a push makes
// its slot stores complete before raising `count`; a thief advances `head`
// only after its slot loads have returned; the owner's capacity check uses
// head/tail.  "Complete before" is drain() over device-coherent accesses
// (see wave.h), not an L2 writeback fence.
//
// Frames come from two pools (64-byte frames; big frames that carry an int32
// buffer).  Each wavefront keeps a free stack per pool in LDS, spills and
// refills fixed-size chunks through a depot of locked bins in global memory,
// and takes never-used frames from a bump pointer.  Capacity exhaustion sets
// a device error word and every wavefront leaves the loop (Sec. 4: overflow
// aborts with a structured report).
#pragma once
#include "layout.h"
#include "tasks.h"
#include "wave.h"

namespace gtap {

constexpr uint32_t kPushSpinLimit = 1u << 16;

constexpr uint32_t kClassCache = 1024;  // children whose DAQ class is kept from the counting pass
constexpr uint32_t kDaqPressure = 2048;  // queued tasks per wavefront above which DAQ runs lowest class first
constexpr uint32_t kLocalFramed = 0xFFFFFFFFu;  // private-stack entry that names a frame (never a job slot)

// Fork descriptor a lane leaves in LDS for the wave-wide child builder:
// {parent frame, job, child kind | big << 7 | d5 << 8, d0..d4}, 32 bytes.
struct alignas(16) ForkDesc {
  uint32_t self, job, ckind_big_d5, d0, d1, d2, d3, d4;
};

struct WaveLds {
  uint32_t stk_s[kStackSmall];
  uint32_t stk_b[kStackBig];
  ForkDesc desc[kWave];
  uint32_t res[kWave];         // parents resumed last iteration, staged this one
  uint32_t next_tid[kWave];    // retained children, by lane, for the next iteration
  uint4 vdesc[kWave * 2];      // images of retained tasks that have no frame
  uint8_t cls[kClassCache];    // DAQ class of child g (counting pass -> build pass)
  uint32_t tail[kMaxQueues];
  uint32_t hint[kMaxQueues];   // 0: own deque q certainly has nothing to pop
  uint32_t head_seen[kMaxQueues];  // last head read by the owner (a lower bound)
  uint32_t qn[kMaxQueues];     // children per class this iteration
  uint32_t qbase[kMaxQueues];  // running rank per class in the build pass
  uint32_t mark[kWave];        // chunk_owner: forking lane + 1 at the slot of its first child
};

// The child-generation descriptor of a fork, as make_child() reads it.
GTAP_DEV Words<6> fork_words(const ForkDesc &dsc) {
  Words<6> d;
  d.w[0] = pack(dsc.d0, dsc.d1);
  d.w[1] = pack(dsc.d2, dsc.d3);
  d.w[2] = pack(dsc.d4, dsc.ckind_big_d5 >> 8);
  return d;
}

// Per-wave statistics: wave-uniform counters kept in registers, added to the
// control block when the wave leaves.
struct WaveCounters {
  uint32_t v[ST_COUNT];
  GTAP_DEV void add(uint32_t i, uint32_t x) { v[i] += x; }
};

GTAP_DEV void raise_error(const Params &p, int32_t code, int32_t pool, uint64_t cap,
                          uint64_t req, uint32_t wave, int32_t job) {
  int32_t zero = 0;
  if (cas_relaxed(&p.ctl->error, &zero, code)) {
    st_relaxed(&p.ctl->err_pool, pool);
    st_relaxed(&p.ctl->err_wave, static_cast<int32_t>(wave));
    st_relaxed(&p.ctl->err_job, job);
    st_relaxed(&p.ctl->err_capacity, cap);
    st_relaxed(&p.ctl->err_requested, req);
  }
}

// ---------------------------------------------------------------------------
// Frame pools.
struct PoolView {
  uint32_t *stk;        // LDS free stack
  int32_t sz;           // stack size (wave-uniform register)
  uint32_t skip;        // allocations left before the depot is probed again
  int32_t net;          // frames handed out minus frames returned (serving accounting)
  uint32_t stk_cap;
  uint32_t chunk;
  DepotBin *bins;
  uint32_t *store;
  uint32_t bincap;      // IDs per bin
  uint64_t *bump;
  uint32_t nframes;
  uint32_t tag;         // kBigBit for the big pool
  int32_t pool_id;
};

GTAP_DEV PoolView small_pool(const Params &p, WaveLds &L) {
  return PoolView{L.stk_s, 0, 0, 0, kStackSmall, kChunkSmall, p.bins_s, p.store_s,
                  p.bincap_s, &p.ctl->bump_small, p.nframes_s, 0u, 0};
}
GTAP_DEV PoolView big_pool(const Params &p, WaveLds &L) {
  return PoolView{L.stk_b, 0, 0, 0, kStackBig, kChunkBig, p.bins_b, p.store_b,
                  p.bincap_b, &p.ctl->bump_big, p.nframes_b, kBigBit, 1};
}

// Lock a depot bin.  Lanes [0, probes) read the chunk counts of consecutive
// bins from the wave's home bin in one round trip; lane 0 then tries the
// locks of the suitable ones in order.  want_room: the bin must have room for
// a chunk, else it must hold one.  Returns the bin and its chunk count, or kNone.
GTAP_DEV uint32_t depot_lock(const PoolView &P, uint32_t me, bool want_room, uint32_t probes,
                             int32_t &nch_out) {
  const int32_t maxchunks = static_cast<int32_t>(P.bincap / P.chunk);
  const uint32_t ln = lane_id();
  uint32_t got = kNone;
  int32_t nch = 0;
  for (uint32_t t0 = 0; t0 < probes && got == kNone; t0 += kWave) {
    const uint32_t t = t0 + ln;
    int32_t seen = want_room ? maxchunks : 0;
    if (t < probes) seen = ld_relaxed(&P.bins[(me + t) % kDepotBins].nchunks);
    uint64_t cand = ballot(t < probes && (want_room ? seen < maxchunks : seen > 0));
    if (ln == 0) {
      while (cand) {
        const uint32_t b = (me + t0 + static_cast<uint32_t>(__ffsll(static_cast<long long>(cand)) - 1)) % kDepotBins;
        cand &= cand - 1;
        DepotBin *bin = P.bins + b;
        int32_t z = 0;
        if (!cas_relaxed(&bin->lock, &z, 1)) continue;
        nch = ld_relaxed(&bin->nchunks);
        if (want_room ? nch < maxchunks : nch > 0) {
          got = b;
          break;
        }
        st_relaxed(&bin->lock, 0);
      }
    }
    got = uniform(got);
  }
  nch_out = uniform(nch);
  return got;
}

GTAP_DEV void depot_unlock(const PoolView &P, uint32_t bin, int32_t nchunks) {
  drain();  // chunk slot accesses complete before the count and lock change
  if (lane_id() == 0) {
    st_relaxed(&P.bins[bin].nchunks, nchunks);
    drain();
    st_relaxed(&P.bins[bin].lock, 0);
  }
}

// Move one chunk from the top of the local stack into a depot bin.  Returns
// false if no bin took it (the IDs then stay on the stack).
GTAP_DEV bool depot_spill(PoolView &P, uint32_t me, WaveCounters &wc) {
  const uint32_t ln = lane_id();
  const int32_t sz = P.sz;
  int32_t nch = 0;
  const uint32_t got = depot_lock(P, me, true, kDepotBins, nch);
  if (got == kNone) return false;
  uint32_t *dst = P.store + static_cast<size_t>(got) * P.bincap + static_cast<size_t>(nch) * P.chunk;
  for (uint32_t i = ln; i < P.chunk; i += kWave) co_st32(dst + i, P.stk[sz - static_cast<int32_t>(P.chunk) + i]);
  depot_unlock(P, got, nch + 1);
  wave_sync();
  P.sz = sz - static_cast<int32_t>(P.chunk);
  wc.add(ST_SPILLS, 1);
  return true;
}

// Pull one chunk from a depot bin onto the local stack.  `all` probes every
// bin, otherwise only a few from the wavefront's home bin.
GTAP_DEV bool depot_refill(PoolView &P, uint32_t me, bool all, WaveCounters &wc) {
  const uint32_t ln = lane_id();
  const int32_t sz = P.sz;
  if (sz + static_cast<int32_t>(P.chunk) > static_cast<int32_t>(P.stk_cap)) return false;
  int32_t nch = 0;
  const uint32_t got = depot_lock(P, me, false, all ? kDepotBins : 8u, nch);
  if (got == kNone) return false;
  const uint32_t *src = P.store + static_cast<size_t>(got) * P.bincap + static_cast<size_t>(nch - 1) * P.chunk;
  for (uint32_t i = ln; i < P.chunk; i += kWave) P.stk[sz + i] = co_ld32(src + i);
  depot_unlock(P, got, nch - 1);
  wave_sync();
  P.sz = sz + static_cast<int32_t>(P.chunk);
  wc.add(ST_REFILLS, 1);
  return true;
}

// Claim `n` fresh frames from the bump pointer; returns the first index or
// kNone when the pool has fewer than n untouched frames left.
GTAP_DEV uint32_t bump_claim(const PoolView &P, uint32_t n) {
  uint32_t base = kNone;
  if (lane_id() == 0) {
    uint64_t cur = ld_relaxed(P.bump);
    while (cur + n <= P.nframes) {
      if (cas_relaxed(P.bump, &cur, cur + n)) {
        base = static_cast<uint32_t>(cur);
        break;
      }
    }
  }
  return uniform(base);
}

// Reserve F frame IDs.  Afterwards ID g (0 <= g < F) is
//   g < taken ? stk[top - 1 - g] : (base + g - taken) | tag,
// with top the stack size before the call.  Returns false on exhaustion.
struct AllocResult {
  int32_t top;
  uint32_t taken;
  uint32_t base;
};

// Every ID handed out by one call must be read (alloc_id) before the next
// allocation from the same pool: the spares of a bump claim are pushed where
// earlier calls' IDs were taken from.
GTAP_DEV bool alloc_frames(const Params &p, PoolView &P, uint32_t me, uint32_t F,
                           AllocResult &r, WaveCounters &wc) {
  P.net += static_cast<int32_t>(F);
  if (static_cast<uint32_t>(P.sz) < F) {
    // Short: recycled frames from nearby depot bins first, unless the last
    // probe found none.
    if (P.skip == 0) {
      while (static_cast<uint32_t>(P.sz) < F) {
        if (!depot_refill(P, me, false, wc)) {
          P.skip = 32;
          break;
        }
      }
    } else {
      --P.skip;
    }
  }
  if (static_cast<uint32_t>(P.sz) >= F) {
    r.top = P.sz;
    r.taken = F;
    r.base = 0;
    P.sz -= static_cast<int32_t>(F);
    return true;
  }
  // Never-used frames: claim F plus a chunk of spares for the local stack.
  uint32_t spare = (P.stk_cap - static_cast<uint32_t>(P.sz)) >= P.chunk ? P.chunk : 0u;
  uint32_t base = bump_claim(P, F + spare);
  if (base == kNone && spare > 0) {
    spare = 0;
    base = bump_claim(P, F);
  }
  if (base != kNone) {
    for (uint32_t i = lane_id(); i < spare; i += kWave) P.stk[P.sz + static_cast<int32_t>(i)] = (base + F + i) | P.tag;
    wave_sync();
    P.sz += static_cast<int32_t>(spare);
    r.top = P.sz;
    r.taken = 0;
    r.base = base;
    return true;
  }
  // The pool is fully touched: reclaim from every bin before giving up.
  while (static_cast<uint32_t>(P.sz) < F) {
    if (!depot_refill(P, me, true, wc)) break;
  }
  if (static_cast<uint32_t>(P.sz) >= F) {
    r.top = P.sz;
    r.taken = F;
    r.base = 0;
    P.sz -= static_cast<int32_t>(F);
    return true;
  }
  if (lane_id() == 0) raise_error(p, -6 /*GTAP_E_CAPACITY*/, P.pool_id, P.nframes, F, me, -1);
  return false;
}

GTAP_DEV uint32_t alloc_id(const PoolView &P, const AllocResult &r, uint32_t g) {
  return g < r.taken ? P.stk[r.top - 1 - static_cast<int32_t>(g)] : ((r.base + (g - r.taken)) | P.tag);
}

// Push the frame of every lane with `mine` set onto its pool's free stack.
GTAP_DEV void free_frames(PoolView &P, uint32_t me, bool mine, uint32_t id, WaveCounters &wc) {
  const uint64_t m = ballot(mine);
  const uint32_t n = __popcll(m);
  if (n == 0) return;
  P.net -= static_cast<int32_t>(n);
  if (P.sz + static_cast<int32_t>(n) > static_cast<int32_t>(P.stk_cap)) {
    if (!depot_spill(P, me, wc)) return;  // no bin took a chunk: these frames are not reused
  }
  const int32_t sz = P.sz;
  if (mine) P.stk[sz + static_cast<int32_t>(rank_below(m))] = id;
  P.sz = sz + static_cast<int32_t>(n);
}

// ---------------------------------------------------------------------------
// Deques.
GTAP_DEV DequeMeta *deque_meta(const Params &p, uint32_t wave, uint32_t q) {
  return p.dq + static_cast<size_t>(wave) * p.Q + q;
}
GTAP_DEV uint32_t *deque_ring(const Params &p, uint32_t wave, uint32_t q) {
  return p.rings + (static_cast<size_t>(wave) * p.Q + q) * p.cap;
}

// PopBatch (Algorithm 2): claim up to 64-cnt IDs from the tail of own deque q.
GTAP_DEV uint32_t pop_batch(const Params &p, WaveLds &L, uint32_t me, uint32_t q, uint32_t cnt,
                            uint32_t &tid, WaveCounters &wc, uint32_t limit = kWave) {
  // Only the owner raises count, so once a pop found it empty (or took all of
  // it) nothing can be popped until the owner pushes again.
  if (L.hint[q] == 0) return 0;
  DequeMeta *m = deque_meta(p, me, q);
  const uint32_t ln = lane_id();
  const int32_t want = static_cast<int32_t>((kWave - cnt) < limit ? (kWave - cnt) : limit);
  int32_t claim = 0;
  uint32_t drained = 0;
  if (ln == 0) {
    int32_t c = ld_relaxed(&m->count);
    for (;;) {
      if (c <= 0) {
        drained = 1;
        break;
      }
      const int32_t take = c < want ? c : want;
      wc.add(ST_RMW, 1);
      if (cas_relaxed(&m->count, &c, c - take)) {
        claim = take;
        drained = (take == c) ? 1u : 0u;
        break;
      }
    }
  }
  claim = uniform(claim);
  if (uniform(drained)) {
    wave_sync();
    if (ln == 0) L.hint[q] = 0;
    wave_sync();
  }
  if (claim == 0) return 0;
  const uint32_t t = L.tail[q] - static_cast<uint32_t>(claim);
  const uint32_t *ring = deque_ring(p, me, q);
  if (ln >= cnt && ln < cnt + static_cast<uint32_t>(claim)) tid = co_ld32(ring + ((t + ln - cnt) & (p.cap - 1)));
  // the slot loads return here: left in flight, they would make the next
  // iteration's first write of this register (the private-stack pop, on
  // the busy path) wait for every memory operation issued before it
  asm volatile("" : "+v"(tid));
  wave_sync();
  if (ln == 0) L.tail[q] = t;
  wave_sync();
  wc.add(ST_POPPED, static_cast<uint32_t>(claim));
  wc.add(ST_POP_BATCHES, 1);
  return static_cast<uint32_t>(claim);
}

// StealBatch.  Lanes [0, steal_probes * Q) each read the count of one
// (random victim, queue) pair in a single round trip; the fullest deque is
// locked, a share of its entries is claimed by CAS on count, the IDs are
// loaded from head, then head advances and the lock is released.  With DAQ
// this takes the victim's fullest queue (Sec. 5.1.3, thread mode).
GTAP_DEV uint32_t steal_batch(const Params &p, uint32_t me, uint32_t &rng, uint32_t cnt, uint32_t &tid,
                              uint32_t &qout, WaveCounters &wc, uint32_t limit = kWave) {
  const uint32_t ln = lane_id();
  wc.add(ST_STEAL_ATTEMPTS, 1);
  const uint32_t probe = ln / p.Q, qi = ln % p.Q;
  const uint32_t base = xorshift32(rng);
  uint32_t v = (base + probe * 0x9E3779B9u) ^ (probe * 0x85EBCA6Bu);
  v ^= v >> 15;
  v *= 0x2C1B3C6Du;
  v ^= v >> 12;
  v = v % (p.nwaves - 1);
  if (v >= me) ++v;
  int32_t c = 0;
  if (probe < p.steal_probes) c = ld_relaxed(&deque_meta(p, v, qi)->count);
  // wave arg-max of the observed counts
  uint32_t key = c > 0 ? ((static_cast<uint32_t>(c < (1 << 24) ? c : (1 << 24) - 1) << 6) | ln) : 0u;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint32_t other = __shfl_xor(key, d, 64);
    key = other > key ? other : key;
  }
  key = uniform(key);
  if (key == 0) return 0;
  const uint32_t win = key & 63u;
  const uint32_t victim = uniform(static_cast<uint32_t>(__shfl(static_cast<int>(v), static_cast<int>(win), 64)));
  const uint32_t q = win % p.Q;
  DequeMeta *m = deque_meta(p, victim, q);
  const int32_t want = static_cast<int32_t>((kWave - cnt) < limit ? (kWave - cnt) : limit);
  int32_t claim = 0;
  uint32_t h = 0;
  if (ln == 0) {
    int32_t z = 0;
    wc.add(ST_RMW, 1);
    if (cas_relaxed(&m->lock, &z, 1)) {
      int32_t cc = static_cast<int32_t>(key >> 6);
      h = ld_relaxed(&m->head);  // stable while we hold the lock
      while (cc > 0) {
        int32_t take = (cc + static_cast<int32_t>(p.steal_div) - 1) / static_cast<int32_t>(p.steal_div);
        take = take < want ? take : want;
        wc.add(ST_RMW, 1);
        if (cas_relaxed(&m->count, &cc, cc - take)) {
          claim = take;
          break;
        }
      }
      if (claim == 0) st_relaxed(&m->lock, 0);
    }
  }
  claim = uniform(claim);
  if (claim == 0) return 0;
  h = uniform(h);
  const uint32_t *ring = deque_ring(p, victim, q);
  if (ln >= cnt && ln < cnt + static_cast<uint32_t>(claim)) tid = co_ld32(ring + ((h + ln - cnt) & (p.cap - 1)));
  drain();  // slot loads returned before head moves past them
  if (ln == 0) {
    st_relaxed(&m->head, h + static_cast<uint32_t>(claim));
    drain();
    st_relaxed(&m->lock, 0);
  }
  qout = q;
  wc.add(ST_STOLEN, static_cast<uint32_t>(claim));
  wc.add(ST_STEAL_BATCHES, 1);
  return static_cast<uint32_t>(claim);
}

// The own deque a wavefront with no tasks starts its next batch from (DAQ):
// the lowest class that can fill a whole wavefront, else the fullest one;
// kNone if every hint says empty.  Low classes hold the tasks nearest to the
// leaves (k-clique: the smallest candidate sets), so draining them first
// keeps the number of live frames close to that of a depth-first order.
// Under queue pressure (the wavefront's class queues hold many tasks) the
// lowest non-empty class is taken instead.
GTAP_DEV uint32_t fullest_own_queue(const Params &p, WaveLds &L, uint32_t me, bool pressure) {
  const uint32_t ln = lane_id();
  int32_t c = 0;
  if (ln < p.Q && L.hint[ln]) c = ld_relaxed(&deque_meta(p, me, ln)->count);
  // only the owner adds to its deques: one read as empty stays empty until it pushes
  wave_sync();
  if (ln < p.Q && L.hint[ln] && c <= 0) L.hint[ln] = 0;
  wave_sync();
  uint32_t rank = 0;
  if (pressure && c > 0) rank = (1u << 23) + (kMaxQueues - ln);
  else if (c >= static_cast<int32_t>(kWave)) rank = (1u << 23) + (kMaxQueues - ln);
  else if (c > 0) rank = static_cast<uint32_t>(c);
  uint32_t key = rank ? ((rank << 6) | ln) : 0u;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint32_t other = __shfl_xor(key, d, 64);
    key = other > key ? other : key;
  }
  key = uniform(key);
  return key == 0 ? kNone : (key & 63u);
}

// Make room for n more IDs in own deque q: head only grows, so a stale copy
// makes the check conservative; reload it only when the check fails.
GTAP_DEV bool ensure_room(const Params &p, WaveLds &L, uint32_t me, uint32_t q, uint32_t n) {
  const uint32_t t = L.tail[q];
  if (t + n - L.head_seen[q] <= p.cap) return true;
  uint32_t ok = 1, h = 0;
  if (lane_id() == 0) {
    DequeMeta *m = deque_meta(p, me, q);
    h = ld_relaxed(&m->head);
    uint32_t spins = 0;
    while (t + n - h > p.cap) {
      if (++spins > kPushSpinLimit) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
      h = ld_relaxed(&m->head);
    }
  }
  ok = uniform(ok);
  h = uniform(h);
  wave_sync();
  if (lane_id() == 0) L.head_seen[q] = h;
  wave_sync();
  if (!ok && lane_id() == 0) raise_error(p, -6 /*GTAP_E_CAPACITY*/, 2, p.cap, n, me, -1);
  return ok != 0;
}

// PushBatch: write n IDs at the tail of own deque q, drain, raise count once
// (the fence and the atomic are paid once per batch, Sec. 5.1.1).
template <class IdFn>
GTAP_DEV bool push_batch(const Params &p, WaveLds &L, uint32_t me, uint32_t q, uint32_t n,
                         IdFn id_of, WaveCounters &wc) {
  if (n == 0) return true;
  if (!ensure_room(p, L, me, q, n)) return false;
  const uint32_t ln = lane_id();
  const uint32_t t = L.tail[q];
  uint32_t *ring = deque_ring(p, me, q);
  for (uint32_t i = ln; i < n; i += kWave) co_st32(ring + ((t + i) & (p.cap - 1)), id_of(i));
  wave_sync();
  if (ln == 0) {
    L.tail[q] = t + n;
    L.hint[q] = 1;
  }
  drain();  // slots (and the frames they name) complete before count rises
  if (ln == 0) fetch_add_relaxed(&deque_meta(p, me, q)->count, static_cast<int32_t>(n));
  wave_sync();
  wc.add(ST_RMW, 1);
  wc.add(ST_PUSHED, n);
  wc.add(ST_PUSH_BATCHES, 1);
  return true;
}

// ---------------------------------------------------------------------------
// Centralised queue (the baseline of the scheduler comparison, Sec. 6.5): one
// FIFO ring for the whole grid.  A push reserves n positions with one atomic
// on tail, writes (position << 32 | ID) into each slot, drains, then raises
// count once.  The slot write is what publishes an entry, so the frame it
// names is drained before it.  A pop claims k <= count by CAS on count (a few attempts per
// call: one while lanes are busy, eight on an empty wavefront; a failed CAS
// means another wavefront claimed), takes positions [head, head + k) with one
// atomic on head and waits until each slot carries its own position (a push
// that reserved earlier may still be writing).  Subtracting first and giving
// back the excess would avoid the retries but can starve: with hundreds of
// pollers the pending give-backs keep the count below zero.  A reservation
// waits while it would reach positions that claims below head - 64 * nwaves
// might still be reading.
GTAP_DEV bool central_reserve(const Params &p, WaveLds &L, uint32_t me, uint32_t n, uint32_t &base) {
  uint32_t b = 0, ok = 1;
  if (lane_id() == 0) {
    b = fetch_add_relaxed(&p.cq->tail, n);
    const uint32_t room = p.ccap - kWave * p.nwaves;
    uint32_t h = L.head_seen[0];
    uint32_t spins = 0;
    while (b + n - h > room) {
      h = ld_relaxed(&p.cq->head);
      if (b + n - h <= room) break;
      if (++spins > kPushSpinLimit) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    L.head_seen[0] = h;
  }
  ok = uniform(ok);
  base = uniform(b);
  wave_sync();
  if (!ok && lane_id() == 0) raise_error(p, -6 /*GTAP_E_CAPACITY*/, 2, p.ccap, n, me, -1);
  return ok != 0;
}

GTAP_DEV void central_put(const Params &p, uint32_t pos, uint32_t id) {
  co_st64(p.cring + (pos & (p.ccap - 1)), (static_cast<uint64_t>(pos) << 32) | id);
}

// The slot write publishes an entry (see central_pop): the frames the IDs name
// must be complete (drained) before the call.
template <class IdFn>
GTAP_DEV bool central_push(const Params &p, WaveLds &L, uint32_t me, uint32_t n, IdFn id_of, WaveCounters &wc) {
  if (n == 0) return true;
  uint32_t b = 0;
  if (!central_reserve(p, L, me, n, b)) return false;
  for (uint32_t i = lane_id(); i < n; i += kWave) central_put(p, b + i, id_of(i));
  drain();
  if (lane_id() == 0) fetch_add_relaxed(&p.cq->count, static_cast<int32_t>(n));
  wc.add(ST_PUSHED, n);
  wc.add(ST_PUSH_BATCHES, 1);
  return true;
}

// Returns the number claimed, or -1 (error raised) if a slot never arrived.
GTAP_DEV int32_t central_pop(const Params &p, uint32_t me, uint32_t cnt, uint32_t &tid, WaveCounters &wc) {
  const uint32_t ln = lane_id();
  const int32_t want = static_cast<int32_t>(kWave - cnt);
  int32_t claim = 0;
  uint32_t pos = 0;
  if (ln == 0) {
    int32_t c = ld_relaxed(&p.cq->count);
    for (uint32_t attempt = cnt == 0 ? 8u : 1u; c > 0 && attempt > 0; --attempt) {
      const int32_t take = c < want ? c : want;
      if (cas_relaxed(&p.cq->count, &c, c - take)) {
        claim = take;
        break;
      }
    }
    if (claim > 0) pos = fetch_add_relaxed(&p.cq->head, static_cast<uint32_t>(claim));
  }
  claim = uniform(claim);
  if (claim == 0) return 0;
  pos = uniform(pos);
  bool lost = false;
  if (ln >= cnt && ln < cnt + static_cast<uint32_t>(claim)) {
    const uint32_t my = pos + (ln - cnt);
    const uint64_t *s = p.cring + (my & (p.ccap - 1));
    uint64_t v = co_ld64(s);
    uint32_t spins = 0;
    while (static_cast<uint32_t>(v >> 32) != my) {
      if (++spins > kPushSpinLimit) {
        lost = true;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      v = co_ld64(s);
    }
    tid = static_cast<uint32_t>(v);
  }
  if (ballot(lost) != 0ull) {
    if (ln == 0) raise_error(p, -6 /*GTAP_E_CAPACITY*/, 2, p.ccap, 0, me, -1);
    return -1;
  }
  wc.add(ST_POPPED, static_cast<uint32_t>(claim));
  wc.add(ST_POP_BATCHES, 1);
  return claim;
}

// ---------------------------------------------------------------------------
// Owner (forking lane) of child g0 + lane, for one 64-child chunk of a
// wavefront's forks: each forking lane whose first child falls in the chunk
// marks that slot, and a prefix maximum over the lanes carries every mark to
// the children after it; `carry` holds the owner of the chunk's first child
// when no mark precedes it (the previous chunk's last owner) and is updated.
// One LDS round trip instead of a binary search over the offsets.  Must be
// called with every lane active.
GTAP_DEV uint32_t chunk_owner(uint32_t *mark, uint32_t nchild, uint32_t off, uint32_t g0, uint32_t &carry) {
  const uint32_t ln = lane_id();
  mark[ln] = 0;
  wave_sync();
  if (nchild > 0 && off >= g0 && off - g0 < kWave) mark[off - g0] = ln + 1;
  wave_sync();
  const uint32_t m = wave_inclusive_max(mark[ln]);
  const uint32_t own = m ? m - 1 : carry;
  carry = __builtin_amdgcn_readlane(own, 63);
  wave_sync();
  return own;
}

// Root frame of job slot j (payload from the job's arguments).
template <uint32_t kExt = 0>
GTAP_DEV void write_root(const Params &p, uint32_t id, uint32_t j) {
  const uint32_t jkind = static_cast<uint32_t>(co_ld64(reinterpret_cast<const uint64_t *>(p.jobs + j)));
  ChildInit c;
  for (uint32_t i = 0; i < kPayloadWords; ++i) c.p[i] = 0;
  uint32_t kind = TK_FIB;
  switch (jkind) {
    case 1:  // fib
      kind = TK_FIB;
      c.p[0] = static_cast<uint32_t>(job_arg(p, j, 0));
      break;
    case 2:  // n-queens: empty board of size n
      kind = TK_NQ;
      c.p[4] = static_cast<uint32_t>(job_arg(p, j, 0));
      break;
    case 3: {  // uts: root id = mix64(seed), depth 0
      kind = TK_UTS;
      const uint64_t rid = mix64(job_arg(p, j, 0));
      const uint64_t thr = job_arg(p, j, 1);
      c.p[0] = static_cast<uint32_t>(rid);
      c.p[1] = static_cast<uint32_t>(rid >> 32);
      c.p[2] = static_cast<uint32_t>(job_arg(p, j, 2)) << 16;
      c.p[3] = static_cast<uint32_t>(thr);
      c.p[4] = static_cast<uint32_t>(thr >> 32);
      break;
    }
    case 4:  // k-clique: the whole vertex range
      kind = TK_KC_RANGE;
      c.p[0] = 0;
      c.p[1] = static_cast<uint32_t>(job_arg(p, j, 2));
      break;
    default:
      break;
  }
  if constexpr (kExt) {
    if constexpr ((kExt & kExtSplit) != 0) {
      if (jkind == 7) {  // k-clique with splitting: the whole vertex range
        kind = TK_KS_RANGE;
        c.p[0] = 0;
        c.p[1] = static_cast<uint32_t>(job_arg(p, j, 2));
      }
    }
    if constexpr ((kExt & kExtLists) != 0) {
      if (jkind == 6) {  // Cilksort: sort the whole array into the key buffer
        kind = TK_SORT;
        c.p[0] = 0;
        c.p[1] = static_cast<uint32_t>(job_arg(p, j, 2));
        c.p[2] = 0;
      }
      // FMM in thread mode: the list-building traversal starts at the pair
      // (root, root); a job whose lists the worklist builds has an empty root
      // (a[0] descriptor, a[1] traversal, a[2] = theta_num | theta_den << 8)
      if (jkind == 5) {
        const uint64_t desc = job_arg(p, j, 0);
        kind = TK_FIB;
        c.p[0] = 0;
        if (job_arg(p, j, 1) == 1) {
          kind = TK_DTT;
          c.p[2] = static_cast<uint32_t>(desc);
          c.p[3] = static_cast<uint32_t>(desc >> 32);
          c.p[4] = static_cast<uint32_t>(job_arg(p, j, 2));
        }
      }
    }
  }
  write_frame(frame_ptr(p, id), kNone, j, state_word(kind, 0, 0), c);
}

// Serving: admit up to 64 jobs the host appended to the admission ring, if the
// in-flight limit and the frame-pool headroom allow.  Admitted roots get
// frames and are pushed to this wave's queue 0.  Returns the number admitted.
GTAP_DEV uint32_t admit_jobs(const Params &p, WaveLds &L, uint32_t me, PoolView &PS, WaveCounters &wc) {
  const uint32_t ln = lane_id();
  uint64_t t = 0;
  int32_t inflight = 0;
  int64_t live = 0, live_b = 0;
  if (ln == 0) {
    t = ld_relaxed(&p.ctl->admitted);
    inflight = ld_relaxed(&p.ctl->jobs_remaining);
    live = ld_relaxed(&p.ctl->live_small);
    live_b = ld_relaxed(&p.ctl->live_big);
  }
  t = uniform64(t);
  inflight = uniform(inflight);
  const uint64_t tk = t + ln;
  const bool ready = sys_ld64(p.ring_seq + (tk % p.ring_cap)) == tk + 1;
  const uint64_t m = ballot(ready);
  uint32_t n = (~m == 0ull) ? kWave : static_cast<uint32_t>(__builtin_ctzll(~m));
  const int32_t allowed = static_cast<int32_t>(p.max_inflight) - inflight;
  if (allowed <= 0) return 0;
  // backpressure: admitted roots go onto this wavefront's deque (and are
  // popped newest first), so admit only while that deque is short
  if (L.tail[0] - L.head_seen[0] > p.cap / 4) {
    uint32_t h = 0;
    if (ln == 0) h = ld_relaxed(&deque_meta(p, me, 0)->head);
    h = uniform(h);
    wave_sync();
    if (ln == 0) L.head_seen[0] = h;
    wave_sync();
    if (L.tail[0] - h > p.cap / 4) return 0;
  }
  if (n > static_cast<uint32_t>(allowed)) n = static_cast<uint32_t>(allowed);
  // admit by free frame-pool memory: keep the headroom free after admitting
  const int64_t ls = static_cast<int64_t>(uniform64(static_cast<uint64_t>(live)));
  const int64_t lb = static_cast<int64_t>(uniform64(static_cast<uint64_t>(live_b)));
  const bool room = ls + static_cast<int64_t>(p.admit_headroom_small) <= static_cast<int64_t>(p.nframes_s) &&
                    (p.nframes_b == 0 || lb + static_cast<int64_t>(p.admit_headroom_big) <= static_cast<int64_t>(p.nframes_b));
  if (n == 0 || !room) return 0;
  uint32_t won = 0;
  if (ln == 0) {
    uint64_t exp = t;
    won = cas_relaxed(&p.ctl->admitted, &exp, t + n) ? 1u : 0u;
  }
  if (!uniform(won)) return 0;
  // copy the job records into the device job table (slot = ticket mod ring_cap)
  for (uint32_t i = ln; i < n; i += kWave) {
    const uint32_t slot = static_cast<uint32_t>((t + i) % p.ring_cap);
    const uint64_t *src = reinterpret_cast<const uint64_t *>(p.ring + slot);
    uint64_t *dst = reinterpret_cast<uint64_t *>(p.jobs + slot);
    for (int w = 0; w < 16; ++w) co_st64(dst + w, sys_ld64(src + w));
    co_st64(&p.jobs[slot].ticket, t + i);
  }
  if (ln == 0) fetch_add_relaxed(&p.ctl->jobs_remaining, static_cast<int32_t>(n));
  AllocResult ar;
  if (!alloc_frames(p, PS, me, n, ar, wc)) return 0;
  wave_sync();
  drain();
  for (uint32_t i = ln; i < n; i += kWave)
    write_root(p, alloc_id(PS, ar, i), static_cast<uint32_t>((t + i) % p.ring_cap));
  drain();
  push_batch(p, L, me, 0, n, [&](uint32_t i) { return alloc_id(PS, ar, i); }, wc);
  wc.add(ST_ADMITTED, n);
  return n;
}

// Capacity of a wavefront's private LDS task stack (task images, 32 bytes
// each): 16 KB per wavefront, 8 KB with eight wavefronts per workgroup (the
// largest power of two with which one such workgroup, 147 KB of LDS, still
// fits a compute unit's 160 KB).
template <int WPB>
struct LocalCap {
  static constexpr uint32_t v = WPB >= 8 ? 256u : 512u;
};

// V selects the queue management (kSchedBatched, kSchedSingle, kSchedCentral;
// kSchedBatchedNoLocal = batched without the private stack) at compile time,
// so the comparison variants add nothing to the scheduler as designed; kExt
// adds extension task sets (kExtLists: the FMM list-building cell pairs and
// their list appends, Cilksort; kExtSplit: split k-clique).
template <int WPB, uint32_t V = kSchedBatched, uint32_t kExt = 0>
__global__ __launch_bounds__(64 * WPB) void thread_sched_kernel(Params p) {
  constexpr bool kCentral = (V == kSchedCentral);
  constexpr bool kSingle = (V == kSchedSingle);
  constexpr bool kNoLocal = (V != kSchedBatched);
  __shared__ WaveLds lds_all[WPB];
  // Private task stack: children a wavefront cannot run in its lanes this
  // iteration stay here as frameless images and are popped (newest first)
  // before the shared deque; only the oldest are exposed to thieves, with
  // frames, when the stack overflows or when the wavefront's deque runs dry
  // while another wavefront is looking for work.
  constexpr uint32_t LC = LocalCap<WPB>::v;
  __shared__ uint4 lstk_all[WPB][2 * LC];
  const uint32_t wv = threadIdx.x >> 6;
  WaveLds &L = lds_all[wv];
  uint4 *lstk = lstk_all[wv];
  uint32_t lbot = 0, ltop = 0;  // wave-uniform: entries [lbot, ltop) mod LC, newest at ltop - 1
  const uint32_t me = blockIdx.x * WPB + wv;
  const uint32_t ln = lane_id();
  const uint64_t deadline = wall_ticks() + p.timeout_ticks;

  WaveCounters wc;
  for (int i = 0; i < static_cast<int>(ST_COUNT); ++i) wc.v[i] = 0;
  uint64_t busy_cycles = 0, idle_cycles = 0;
  uint64_t data_words = 0;  // this lane's task-data words (summed over the wave on exit)
  if (ln == 0) {
    for (uint32_t q = 0; q < kMaxQueues; ++q) {
      L.tail[q] = 0;
      L.hint[q] = 0;
      L.head_seen[q] = 0;
    }
  }
  wave_sync();

  PoolView PS = small_pool(p, L);
  PoolView PB = big_pool(p, L);
  uint32_t rng = 0x9E3779B9u ^ (me * 0x85EBCA6Bu + 1u);

  uint32_t cnt = 0;
  uint32_t tid = kNone;
  uint32_t npend = 0;    // parents resumed in the last iteration (IDs in L.res)
  uint32_t cur_q = 0;    // DAQ class of the batch on the lanes
  bool daq_pressure = false;  // DAQ: own class queues hold more than kDaqPressure tasks

  // Root admission: job j goes to wave j mod P (the paper's grid leader
  // enqueues the single root; with many jobs every wave seeds its share).
  // Roots get frames.
  {
    const uint32_t nroots = me < p.njobs ? (p.njobs - me + p.nwaves - 1) / p.nwaves : 0u;
    AllocResult ar{};
    const bool ok = alloc_frames(p, PS, me, nroots, ar, wc);
    if (ok && nroots > 0) {
      wave_sync();
      for (uint32_t g = ln; g < nroots; g += kWave) write_root<kExt>(p, alloc_id(PS, ar, g), me + g * p.nwaves);
      drain();
      const uint32_t keep = nroots < kWave ? nroots : kWave;
      if (ln < keep) tid = alloc_id(PS, ar, ln);
      cnt = keep;
      auto root_id = [&](uint32_t i) { return alloc_id(PS, ar, keep + i); };
      if constexpr (kCentral) central_push(p, L, me, nroots - keep, root_id, wc);
      else push_batch(p, L, me, 0, nroots - keep, root_id, wc);
    }
  }

  uint32_t idle = 0;
  uint32_t iter = 0;
  bool hungry = false;  // counted in the control block's hungry-wavefront hint
  bool tcont = false;  // this lane's task is a resumed parent (runs its continuation)
  fmm::ListChunks lchunks{nullptr, {0, 0}, {fmm::kListChunk, fmm::kListChunk}};  // FMM list traversal only
  uint64_t t_loop = clock64();
  // Join RMWs of the last busy iteration.  Their old values are examined in
  // the next iteration, after its tasks ran, so the RMW latency overlaps that
  // work; an iteration that publishes nothing to a shared deque ends without
  // a drain, and the drain in examine() orders its writes before the next
  // completion RMWs.
  bool pend_any = false;
  bool pend_tail = false;
  // frame words of the continuation this lane runs next iteration, loaded as
  // soon as the parent is known to resume (one iteration ahead)
  TaskImage cpre{0, 0, 0, 0};
  bool cpre_ok = false;
  int64_t pend_old = 0;
  uint32_t pend_len = 0, pend_par = kNone;
  auto examine = [&]() {
    drain();
    // both halves of the RMW result stay allocated until here (only the low
    // half is examined; a register reused for anything else before this point
    // would have to wait for the RMW first)
    asm volatile("" : : "v"(pend_old));
    const bool resumed = pend_tail && (static_cast<uint64_t>(pend_old) & kJoinMask) == pend_len;
    const uint64_t m_res = ballot(resumed);
    wave_sync();
    if (resumed) L.res[rank_below(m_res)] = pend_par;
    npend = __popcll(m_res);
    wave_sync();
    pend_any = false;
    pend_tail = false;
  };
  for (;;) {
    // ---- serving: a few waves admit newly submitted jobs ----
    // (any other wavefront also admits when it has been idle for a while, so
    // a burst of arrivals spreads over the grid instead of over eight deques)
    if (p.serving && (me < kAdmitWaves ? (cnt == 0 || (iter & 15u) == 0) : (cnt == 0 && (idle & 7u) == 4u)))
      admit_jobs(p, L, me, PS, wc);
    // ---- acquire work ----
    // Parents resumed by the last iteration's RMWs are normally staged with
    // this iteration's children; with no lanes busy they run right away.
    if (cnt == 0 && pend_any) examine();
    if (cnt == 0 && npend > 0) {
      if (ln < npend) {
        tid = L.res[ln];
        tcont = true;
      }
      cnt = npend;
      npend = 0;
    }
    // popped and stolen tasks are children with frames (resume point 0); a
    // batch is topped up from the queue of its class, an empty wavefront
    // starts from its fullest queue
    const uint32_t cnt0 = cnt;
    if (p.Q == 1 && cnt < kWave && ltop != lbot) {
      const uint32_t have = ltop - lbot;
      const uint32_t take = (kWave - cnt) < have ? (kWave - cnt) : have;
      if (ln >= cnt && ln < cnt + take) {
        const uint32_t e = (ltop - 1 - (ln - cnt)) & (LC - 1);
        const uint4 a = lstk[2 * e];
        if (a.y == kLocalFramed) {
          tid = a.x;  // a task with a frame (it carries a buffer)
        } else {
          L.vdesc[2 * ln] = a;
          L.vdesc[2 * ln + 1] = lstk[2 * e + 1];
          tid = kNone;
        }
      }
      wave_sync();
      ltop -= take;
      cnt += take;
    }
    if constexpr (kCentral) {
      if (cnt < kWave) {
        const int32_t got = central_pop(p, me, cnt, tid, wc);
        if (got < 0) break;
        cnt += static_cast<uint32_t>(got);
      }
    } else if constexpr (kSingle) {
      // non-batched: one task per pop, up to the free lanes
      while (cnt < kWave) {
        const uint32_t got = pop_batch(p, L, me, 0, cnt, tid, wc, 1);
        if (got == 0) break;
        cnt += got;
      }
    } else if (cnt < kWave) {
      uint32_t qp = cur_q;
      if (cnt == 0 && p.Q > 1) {
        qp = fullest_own_queue(p, L, me, daq_pressure);
        if (qp != kNone) cur_q = qp;
      }
      if (qp != kNone) cnt += pop_batch(p, L, me, qp, cnt, tid, wc);
    }
    // DAQ: a wavefront that still holds tasks in its own class queues runs a
    // partial batch rather than stealing, so it finishes its own subtrees
    // first (stealing new work instead grows the pending frontier breadth-first)
    const bool own_left = p.Q > 1 && cnt > 0 && ballot(ln < p.Q && L.hint[ln] != 0) != 0ull;
    if constexpr (kSingle) {
      // non-batched: one task per steal, until one fails or the lanes are full
      if (cnt < p.steal_below && p.nwaves > 1) {
        while (cnt < kWave) {
          uint32_t qs = 0;
          const uint32_t got = steal_batch(p, me, rng, cnt, tid, qs, wc, 1);
          if (got == 0) break;
          cnt += got;
        }
      }
    } else if (!kCentral && cnt < p.steal_below && p.nwaves > 1 && !own_left) {
      uint32_t qs = cur_q;
      const uint32_t got = steal_batch(p, me, rng, cnt, tid, qs, wc);
      if (got > 0 && cnt == 0) cur_q = qs;
      cnt += got;
    }
    if (ln >= cnt0) tcont = false;
    if (cnt == 0) {
      ++idle;
      wc.add(ST_IDLE, 1);
      if (!hungry) {
        if (ln == 0) fetch_add_relaxed(&p.ctl->hungry, 1);
        hungry = true;
      }
      // termination: every root completed (the implicit join at each task's
      // end makes a root the last task of its job), an error, or the watchdog
      uint32_t stop = 0;
      if ((idle & 3u) == 1u && ln == 0) {
        // batch: every root completed; serving: stop requested and nothing in flight
        const bool drained_jobs = ld_relaxed(&p.ctl->jobs_remaining) <= 0 &&
                                  (!p.serving || ((idle & 15u) == 1u && sys_ld32i(p.stop_host) != 0));
        if (drained_jobs || ld_relaxed(&p.ctl->error) != 0) stop = 1;
        else if (wall_ticks() > deadline) {
          raise_error(p, -8 /*GTAP_E_TIMEOUT*/, 3, p.timeout_ticks, 0, me, -1);
          stop = 1;
        }
      }
      if (uniform(stop)) break;
      if (p.serving && ln == 0) {
        if (PS.net) fetch_add_relaxed(&p.ctl->live_small, static_cast<int64_t>(PS.net));
        if (PB.net) fetch_add_relaxed(&p.ctl->live_big, static_cast<int64_t>(PB.net));
      }
      PS.net = 0;
      PB.net = 0;
      backoff_sleep(idle);
      const uint64_t now = clock64();
      idle_cycles += now - t_loop;
      t_loop = now;
      continue;
    }
    idle = 0;
    if (hungry) {
      if (ln == 0) fetch_add_relaxed(&p.ctl->hungry, -1);
      hungry = false;
    }
    ++iter;
    if (p.Q > 1 && (iter & 7u) == 0) {
      // DAQ queue pressure: tasks waiting in this wavefront's class queues
      int32_t c = 0;
      if (ln < p.Q) c = ld_relaxed(&deque_meta(p, me, ln)->count);
      const uint32_t tot = static_cast<uint32_t>(
          __builtin_amdgcn_readlane(static_cast<int>(wave_inclusive_sum(c > 0 ? static_cast<uint32_t>(c) : 0u)), 63));
      daq_pressure = tot > kDaqPressure;
    }
    if ((iter & 63u) == 0) {
      uint32_t stop = 0;
      if (ln == 0) {
        if (ld_relaxed(&p.ctl->error) != 0) stop = 1;
        else if (wall_ticks() > deadline) {
          raise_error(p, -8 /*GTAP_E_TIMEOUT*/, 3, p.timeout_ticks, 0, me, -1);
          stop = 1;
        }
      }
      if (uniform(stop)) break;
    }
    wc.add(ST_ITERS, 1);

    // ---- execute one task per lane ----
    // (a lane about to load a frame this wavefront may have written in the
    // last iteration -- a retained or privately stacked child with a frame --
    // waits for those writes)
    if (pend_any && ballot(ln < cnt && tid != kNone && !tcont) != 0ull) drain();
    Outcome o;
    o.type = OUT_NONE;
    o.nchild = 0;
    o.big = 0;
    o.first = 0;
    o.words = 0;
    for (int i = 0; i < 6; ++i) o.d[i] = 0;
    if constexpr (kExt) o.emit = 0;
    if (ln < cnt) {
      TaskImage img;
      if (tid == kNone) {
        const uint4 a = L.vdesc[2 * ln], b = L.vdesc[2 * ln + 1];
        img = TaskImage{pack(a.x, a.y), pack(a.z, a.w), pack(b.x, b.y), pack(b.z, b.w)};
      } else if (tcont) {
        img = cpre_ok ? cpre : load_continuation(p, tid);
      } else {
        img = load_image(p, tid);
      }
      exec_task<kExt>(p, tid, img, o);
    }
    if constexpr ((kExt & kExtLists) != 0) {
      // FMM list traversal: accepted pairs and leaf pairs go to their lists,
      // through this wavefront's chunks of them
      const bool em = o.type == OUT_DONE && o.emit != 0;
      if (ballot(em) != 0ull) {
        fmm::FmmDesc *D = reinterpret_cast<fmm::FmmDesc *>(pack(o.d[3], o.d[4]));
        const uint64_t pair = (static_cast<uint64_t>(o.d[0]) << 32) | o.d[1];
        fmm::chunks_append(lchunks, D, 0, em && o.emit == 1, pair);
        fmm::chunks_append(lchunks, D, 1, em && o.emit == 2, pair);
      }
    }
    data_words += o.words;
    const uint32_t nfirst = __popcll(ballot(o.first != 0));
    wc.add(ST_TASKS, nfirst);
    wc.add(ST_CONTS, cnt - nfirst);

    // ---- completions ----
    // A child's completion adds its result to the parent's join word and
    // decrements the waiting-child count in the same RMW; the child that
    // brings the count to zero resumes the parent (Sec. 5.1.2).  Siblings that
    // completed on adjacent lanes are summed first (a prefix sum over the wave
    // minus the prefix before the run's first lane), so each parent receives
    // one RMW per wavefront.  The RMW's old value is examined in the next
    // iteration, and the parents it resumed are staged with that iteration's
    // children.
    const bool done = (o.type == OUT_DONE);
    const bool to_parent = done && o.parent != kNone;
    const bool root_done = done && o.parent == kNone;
    if (root_done) {
      JobSlot &J = p.jobs[o.job];
      const uint64_t now = wall_ticks();
      st_relaxed(&J.result, o.value);
      st_relaxed(&J.t_done, now);
      st_relaxed(&J.done, 1u);
      if (p.serving) {
        HostCompletion *h = p.done_host + o.job;
        sys_st64(reinterpret_cast<uint64_t *>(&h->result), static_cast<uint64_t>(o.value));
        sys_st64(&h->t_done, now);
      }
    }
    const uint32_t par = to_parent ? o.parent : kNone;
    const uint32_t prev_par = wave_from_below(par, kNone);
    const uint32_t next_par = wave_from_above(par, kNone);
    const bool head = !to_parent || prev_par != par;
    const bool tail = to_parent && next_par != par;
    const uint32_t hidx = wave_inclusive_max(head ? ln : 0u);
    const uint64_t pre = wave_inclusive_sum64(to_parent ? static_cast<uint64_t>(o.value) : 0ull);
    const uint32_t src = hidx > 0 ? hidx - 1 : 0;
    const uint64_t pre_lo = static_cast<uint32_t>(__shfl(static_cast<int>(static_cast<uint32_t>(pre)), static_cast<int>(src), 64));
    const uint64_t pre_hi = static_cast<uint32_t>(__shfl(static_cast<int>(static_cast<uint32_t>(pre >> 32)), static_cast<int>(src), 64));
    const uint64_t before = hidx > 0 ? (pre_lo | (pre_hi << 32)) : 0ull;
    const int64_t run_val = static_cast<int64_t>(pre - before);
    const uint32_t run_len = ln - hidx + 1;
    // the previous iteration's RMW results (its writes complete before these RMWs)
    cpre_ok = false;
    if (pend_any) {
      examine();
      // the parents it resumed run next iteration on lanes [0, npend): their
      // frames are fetched now
      if (ln < npend) {
        cpre = load_continuation(p, L.res[ln]);
        cpre_ok = true;
      }
    }
    if constexpr (kExt) {
      // Cilksort keys, rows of a vertex's k-clique bit matrix: what a task
      // wrote is complete before its completion can resume the parent that
      // hands it to the next tasks
      if (ballot(done && (o.kind == TK_SORT || o.kind == TK_MERGE || o.kind == TK_KS_ROW)) != 0ull) drain();
    }
    const int64_t lim = static_cast<int64_t>(1) << kSmallValueBits;
    const bool big_val = tail && (run_val >= lim || run_val <= -lim);
    const uint64_t big_lanes = ballot(big_val);
    if (big_lanes) {
      if (big_val) fetch_add_relaxed(bigacc_ptr(frame_ptr(p, o.parent)), run_val);
      drain();  // the large result is in place before the count can reach zero
    }
    wc.add(ST_RMW, static_cast<uint32_t>(__popcll(ballot(tail))) + static_cast<uint32_t>(__popcll(big_lanes)));
    // The RMW returns straight into the register examine() reads next
    // iteration (pend_old is dead from here on): a register copy of the
    // result at the end of the iteration would make the wavefront wait for
    // the RMW, and every store issued after it, there.
    if (tail) {
      const int64_t delta = (big_val ? 0 : run_val * (static_cast<int64_t>(1) << kJoinBits)) -
                            static_cast<int64_t>(run_len);
      pend_old = fetch_add_relaxed(join_ptr(frame_ptr(p, o.parent)), delta);
    }
    const uint32_t pend_par_next = o.parent;
    if (ballot(root_done)) {
      drain();  // the job's result is in place before the run can end or the host sees it
      if (root_done && p.serving) sys_st64(&p.done_host[o.job].done, co_ld64(&p.jobs[o.job].ticket) + 1);
      if (root_done) fetch_add_relaxed(&p.ctl->jobs_remaining, -1);
    }
    // completed tasks that had frames release them
    free_frames(PS, me, done && tid != kNone && !(tid & kBigBit), tid, wc);
    free_frames(PB, me, done && tid != kNone && (tid & kBigBit), tid, wc);

    // ---- forks ----
    if (ballot(o.type == OUT_FORK && o.nchild > kMaxChildren)) {
      if (ln == 0) raise_error(p, -6 /*GTAP_E_CAPACITY*/, 4, kMaxChildren, 0, me, -1);
      break;
    }
    const bool fork = (o.type == OUT_FORK);
    const bool need_self = fork && tid == kNone;  // a frameless task suspends: give it a frame
    uint32_t F = 0;
    const uint32_t off = wave_exclusive_scan(fork ? o.nchild : 0u, &F);
    const uint64_t m_self = ballot(need_self);
    const uint32_t nres = npend;
    AllocResult aself;
    if (!alloc_frames(p, PS, me, __popcll(m_self), aself, wc)) break;
    wave_sync();
    wc.add(ST_SPAWNS, F);
    if (fork) {
      // suspend at the join: resume point 1, count = #children, sums 0
      const uint32_t self = need_self ? alloc_id(PS, aself, rank_below(m_self)) : tid;
      uint32_t *f = frame_ptr(p, self);
      if (need_self) co_st64(frame64(f), pack(o.parent, o.job));
      if constexpr (kExt) {
        // Cilksort sorts and k-clique vertices resume twice and read their
        // arguments from the frame
        co_st32(f + FW_STATE, state_word(o.kind, o.pc_next, 0));
        if (need_self && (o.kind == TK_SORT || o.kind == TK_KS_VERTEX)) {
          co_st32(f + FW_P0, o.d[0]);
          co_st32(f + FW_P0 + 1, o.d[1]);
          co_st32(f + FW_P0 + 2, o.d[2]);
        }
      } else {
        co_st32(f + FW_STATE, state_word(o.kind, 1, 0));
      }
      st_relaxed(bigacc_ptr(f), static_cast<int64_t>(0));
      st_relaxed(join_ptr(f), static_cast<int64_t>(o.nchild));
      L.desc[ln] = ForkDesc{self, o.job, o.ckind | (o.big << 7) | (o.d[5] << 8),
                            o.d[0], o.d[1], o.d[2], o.d[3], o.d[4]};
    }
    if (ln < kMaxQueues) L.qn[ln] = (ln == 0) ? F : 0u;
    wave_sync();

    // ---- DAQ counting pass: children per class; the fullest class is kept ----
    uint32_t R = 0;
    if (p.Q > 1 && F > 0) {
      if (ln < kMaxQueues) L.qn[ln] = 0;
      wave_sync();
      uint32_t own_carry = 0;
      for (uint32_t g0 = 0; g0 < F; g0 += kWave) {
        const uint32_t g = g0 + ln;
        const uint32_t own = chunk_owner(L.mark, fork ? o.nchild : 0u, off, g0, own_carry);
        const uint32_t own_off = static_cast<uint32_t>(__shfl(static_cast<int>(off), static_cast<int>(own), 64));
        uint32_t c = kNone;
        if (g < F) {
          const ForkDesc dsc = L.desc[own];
          const Words<6> d = fork_words(dsc);
          ChildInit ci;
          make_child<kExt>(dsc.ckind_big_d5 & 0x7Fu, d, g - own_off, ci);
          c = child_class<kExt>(p, dsc.job, dsc.ckind_big_d5 & 0x7Fu, ci);
          if (g < kClassCache) L.cls[g] = static_cast<uint8_t>(c);
        }
        for (uint32_t qq = 0; qq < p.Q; ++qq) {
          const uint32_t k = __popcll(ballot(c == qq));
          if (ln == 0) L.qn[qq] += k;
        }
      }
      wave_sync();
      uint32_t best = 0;
      if (daq_pressure) {
        // queue pressure: keep the lowest class present (nearest the leaves)
        while (best + 1 < p.Q && L.qn[best] == 0) ++best;
      } else {
        for (uint32_t qq = 1; qq < p.Q; ++qq)
          if (L.qn[qq] > L.qn[best]) best = qq;
      }
      R = uniform(best);
    }
    const uint32_t nR = L.qn[R];
    const uint32_t keep = (kWave - nres) < nR ? (kWave - nres) : nR;
    // ---- private stack (one queue): small children beyond the lanes stay in
    // LDS; the oldest entries are exposed when it would overflow, or when the
    // wavefront's own deque has run dry and some wavefront has found no work
    // (thieves then find some) ----
    const bool use_local = !kNoLocal && (p.Q == 1);
    uint32_t E = 0, direct = 0, nsmall = 0;
    if (use_local) {
      nsmall = F - keep;  // every child beyond the lanes is a candidate
      const uint32_t have = ltop - lbot;
      uint32_t ex = (have + nsmall > LC) ? (have + nsmall - LC) : 0u;
      if (ex > have) ex = have;
      if ((iter & 7u) == 0 && have >= 2 * kWave) {
        // half the stack goes to the deque when it runs low and some
        // wavefront is looking for work (both words read in one round trip)
        int32_t c = 0;
        if (ln == 0) c = ld_relaxed(&deque_meta(p, me, 0)->count);
        if (ln == 1) c = ld_relaxed(&p.ctl->hungry);
        const int32_t own = __builtin_amdgcn_readlane(c, 0), seekers = __builtin_amdgcn_readlane(c, 1);
        if (own < static_cast<int32_t>(kWave) && seekers > 0 && have / 2 > ex) ex = have / 2;
      }
      E = ex;
      const uint32_t free_slots = LC - (have - E);
      direct = nsmall > free_slots ? nsmall - free_slots : 0u;
    }
    const uint32_t nglob = use_local ? (F - keep) - (nsmall - direct) + E : 0u;
    bool room = true;
    uint32_t cbase = 0;  // centralised queue: first reserved position
    if constexpr (kCentral) {
      const uint32_t n = L.qn[0] - keep;
      if (n > 0) room = central_reserve(p, L, me, n, cbase);
    } else {
      for (uint32_t qq = 0; qq < p.Q; ++qq) {
        const uint32_t n = use_local ? nglob : L.qn[qq] - (qq == R ? keep : 0u);
        if (n > 0) room = room && ensure_room(p, L, me, qq, n);
      }
    }
    if (!room) break;
    if (E > 0) {
      // the oldest local entries take the first ring slots; frameless ones
      // get frames first
      bool ok = true;
      for (uint32_t i0 = 0; i0 < E && ok; i0 += kWave) {
        const uint32_t i = i0 + ln;
        const bool act = i < E;
        uint4 a = make_uint4(0, 0, 0, 0), b = a;
        if (act) {
          const uint32_t e = (lbot + i) & (LC - 1);
          a = lstk[2 * e];
          b = lstk[2 * e + 1];
        }
        const bool framed = act && a.y == kLocalFramed;
        const uint64_t m_f = ballot(act && !framed);
        AllocResult ae;
        ok = alloc_frames(p, PS, me, __popcll(m_f), ae, wc);
        if (!ok) break;
        wave_sync();
        if (act) {
          uint32_t cid = a.x;
          if (!framed) {
            cid = alloc_id(PS, ae, rank_below(m_f));
            ChildInit ci;
            ci.p[0] = a.w;
            ci.p[1] = b.x;
            ci.p[2] = b.y;
            ci.p[3] = b.z;
            ci.p[4] = b.w;
            write_frame(frame_ptr(p, cid), a.x, a.y, a.z, ci);
          }
          co_st32(deque_ring(p, me, 0) + ((L.tail[0] + i) & (p.cap - 1)), cid);
        }
      }
      if (!ok) break;
      wave_sync();
      lbot += E;
    }
    uint32_t lbase = 0, gbase = E;

    // ---- build pass: children are retained (class R, first `keep` of them)
    // or written to a frame and placed in their class's deque ----
    if (ln < kMaxQueues) L.qbase[ln] = 0;
    wave_sync();
    bool alloc_ok = true;
    uint32_t own_carry = 0;
    for (uint32_t g0 = 0; g0 < F; g0 += kWave) {
      const uint32_t g = g0 + ln;
      const bool act = g < F;
      const uint32_t own = chunk_owner(L.mark, fork ? o.nchild : 0u, off, g0, own_carry);
      const uint32_t own_off = static_cast<uint32_t>(__shfl(static_cast<int>(off), static_cast<int>(own), 64));
      uint32_t j = 0, c = 0;
      ForkDesc dsc{};
      ChildInit ci;
      if (act) {
        j = g - own_off;
        dsc = L.desc[own];
        const Words<6> d = fork_words(dsc);
        make_child<kExt>(dsc.ckind_big_d5 & 0x7Fu, d, j, ci);
        if (p.Q > 1) c = g < kClassCache ? L.cls[g] : child_class<kExt>(p, dsc.job, dsc.ckind_big_d5 & 0x7Fu, ci);
      }
      const bool big = act && (dsc.ckind_big_d5 & 0x80u);
      // rank of this child within its class
      uint32_t rank = g;
      if (p.Q > 1) {
        for (uint32_t qq = 0; qq < p.Q; ++qq) {
          const uint64_t m = ballot(act && c == qq);
          if (act && c == qq) rank = L.qbase[qq] + rank_below(m);
          wave_sync();
          if (ln == 0) L.qbase[qq] += __popcll(m);
          wave_sync();
        }
      }
      const bool keep_me = act && c == R && rank < keep;
      uint32_t cput_pos = 0, cput_id = kNone;
      // small children beyond the lanes: the first `direct` go to the shared
      // deque, the rest onto the private stack
      const bool cand = use_local && act && !keep_me;
      const uint64_t m_c = ballot(cand);
      const uint32_t lr = lbase + rank_below(m_c);
      lbase += __popcll(m_c);
      const bool to_local = cand && lr >= direct;
      const uint64_t m_g = ballot(act && !keep_me && !to_local);
      const uint32_t gpos = gbase + rank_below(m_g);
      gbase += __popcll(m_g);
      const bool frameless = keep_me && !big;
      const uint64_t m_s = ballot(act && !big && !keep_me && !to_local);
      const bool local_framed = to_local && big;
      const uint64_t m_b = ballot(big);
      AllocResult as_, ab_;
      alloc_ok = alloc_frames(p, PS, me, __popcll(m_s), as_, wc) && alloc_frames(p, PB, me, __popcll(m_b), ab_, wc);
      if (!alloc_ok) break;
      wave_sync();
      if (act) {
        const uint32_t ck = dsc.ckind_big_d5 & 0x7Fu;
        const uint32_t st = state_word(ck, 0, c);
        uint32_t cid = kNone;
        if (local_framed) {
          cid = alloc_id(PB, ab_, rank_below(m_b));
          write_frame(frame_ptr(p, cid), dsc.self, dsc.job, st, ci);
          const uint32_t e = (ltop + lr - direct) & (LC - 1);
          lstk[2 * e] = make_uint4(cid, kLocalFramed, 0, 0);
        } else if (to_local) {
          const uint32_t e = (ltop + lr - direct) & (LC - 1);
          lstk[2 * e] = make_uint4(dsc.self, dsc.job, st, ci.p[0]);
          lstk[2 * e + 1] = make_uint4(ci.p[1], ci.p[2], ci.p[3], ci.p[4]);
        } else if (frameless) {
          uint4 *v = L.vdesc + 2 * (nres + rank);
          v[0] = make_uint4(dsc.self, dsc.job, st, ci.p[0]);
          v[1] = make_uint4(ci.p[1], ci.p[2], ci.p[3], ci.p[4]);
        } else {
          cid = big ? alloc_id(PB, ab_, rank_below(m_b)) : alloc_id(PS, as_, rank_below(m_s));
          write_frame(frame_ptr(p, cid), dsc.self, dsc.job, st, ci);
        }
        if (keep_me) {
          L.next_tid[nres + rank] = cid;
        } else if (!to_local) {
          const uint32_t pos = use_local ? gpos : rank - (c == R ? keep : 0u);
          if constexpr (kCentral) {
            cput_pos = cbase + pos;
            cput_id = cid;
          } else {
            co_st32(deque_ring(p, me, c) + ((L.tail[c] + pos) & (p.cap - 1)), cid);
          }
        }
      }
      // centralised queue: a claim may cover positions of pushes that have not
      // raised count yet, so the slot write itself publishes the entry -- the
      // frames it names complete first
      if constexpr (kCentral) {
        if (ballot(cput_id != kNone) != 0ull) {
          drain();
          if (cput_id != kNone) central_put(p, cput_pos, cput_id);
        }
      }
    }
    if (!alloc_ok) break;
    if (use_local) {
      ltop += nsmall - direct;
      wc.add(ST_LOCAL, nsmall - direct);
    }
    {
      const uint32_t qq = ln;
      const uint32_t n = (qq < p.Q) ? (use_local ? nglob : L.qn[qq] - (qq == R ? keep : 0u)) : 0u;
      // frames and ring slots written this iteration are complete before any
      // of them is published
      const uint64_t pushing = ballot(n > 0);
      if (pushing != 0ull) drain();
      if (n > 0)
        fetch_add_relaxed(kCentral ? &p.cq->count : &deque_meta(p, me, qq)->count, static_cast<int32_t>(n));
      wc.add(ST_RMW, static_cast<uint32_t>(__popcll(pushing)));
      wave_sync();
      if (n > 0) {
        L.tail[qq] += n;
        L.hint[qq] = 1;
      }
      const uint32_t npushed = uniform(static_cast<uint32_t>(__builtin_amdgcn_readlane(
          static_cast<int>(wave_inclusive_sum(n)), 63)));
      if (npushed > 0) {
        wc.add(ST_PUSHED, npushed);
        wc.add(ST_PUSH_BATCHES, 1);
      }
    }
    wave_sync();

    // ---- next batch: resumed parents, then the retained children ----
    if (ln < nres) tid = L.res[ln];
    else if (ln < nres + keep) tid = L.next_tid[ln];
    else tid = kNone;
    tcont = ln < nres;
    cnt = nres + keep;
    if (keep > 0) cur_q = R;
    npend = 0;  // staged above
    pend_any = true;
    pend_tail = tail;
    pend_len = run_len;
    pend_par = pend_par_next;
    // serving: live-frame deltas reach the shared counters in batches (two
    // same-address atomics per wavefront per iteration would serialise)
    if (p.serving && ((iter & 63u) == 0 || PS.net > 1024 || PS.net < -1024 || PB.net > 256 || PB.net < -256)) {
      if (ln == 0) {
        if (PS.net) fetch_add_relaxed(&p.ctl->live_small, static_cast<int64_t>(PS.net));
        if (PB.net) fetch_add_relaxed(&p.ctl->live_big, static_cast<int64_t>(PB.net));
      }
      PS.net = 0;
      PB.net = 0;
    }
    const uint64_t now = clock64();
    busy_cycles += now - t_loop;
    t_loop = now;
  }

  if constexpr ((kExt & kExtLists) != 0) fmm::chunks_close(lchunks);
  // ---- flush counters ----
  const uint64_t wave_words = wave_inclusive_sum64(data_words);
  const uint64_t words_total = readlane64(wave_words, 63);
  if (ln == 0) {
    if (words_total) fetch_add_relaxed(&p.ctl->stats[ST_DATA_WORDS], words_total);
    for (int i = 0; i < static_cast<int>(ST_COUNT); ++i)
      if (wc.v[i]) fetch_add_relaxed(&p.ctl->stats[i], static_cast<uint64_t>(wc.v[i]));
    if (busy_cycles) fetch_add_relaxed(&p.ctl->stats[ST_BUSY_CYCLES], busy_cycles);
    if (idle_cycles) fetch_add_relaxed(&p.ctl->stats[ST_IDLE_CYCLES], idle_cycles);
  }
}

}  // namespace gtap
