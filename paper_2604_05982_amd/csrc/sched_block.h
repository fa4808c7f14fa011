// sched_block.h -- block-mode persistent scheduler: one task per workgroup.
//
// Block mode (GTaP Sec. 4.3, 5.1.3): every thread of a workgroup runs the same
// task cooperatively.  Each workgroup owns one Chase-Lev deque (Chase and Lev,
// SPAA 2005): the owner pushes and pops at the bottom, thieves take one task
// at a time from the top with a CAS.  Thread 0 runs the queue operations and
// broadcasts the task through LDS; wavefront 0 allocates and frees frames with
// the same pools and depot as thread mode; the body runs on all threads.
//
// Fib and UTS tasks use the frames, join words and implicit join at task
// return of thread mode.  FMM cell-pair tasks have no result and nothing to
// do after their children, so they are counted instead: a job keeps the
// number of its outstanding cell-pair tasks, a workgroup accumulates
// (children created - tasks completed) and adds it to the job's counter at
// once when positive, lazily when negative.  Every workgroup's unadded
// amount is thus <= 0, the counter never falls below the true outstanding
// count, and it reaches zero exactly when the job is done.  Their children
// stay as 32-byte images on a private LDS stack and are run newest first;
// only the oldest get frames and go to the Chase-Lev deque, when the stack
// overflows or the deque has run dry.
//
// Memory ordering: every cross-workgroup word is accessed device-coherently
// and drain() waits for completion.  The owner's bottom decrement is an atomic
// exchange performed before top is read; a thief reads top, then bottom, then
// the slot, each after the previous access completed, and claims the slot by
// CAS on top.
#pragma once
#include "fmm.h"
#include "sched_thread.h"
#include "tasks.h"

namespace gtap {

struct alignas(128) ClDeque {
  int64_t top;      // thieves' end: only grows, advanced by CAS
  int64_t bottom;   // owner's end
  int64_t pad[14];
};
static_assert(sizeof(ClDeque) == sizeof(DequeMeta), "block deques reuse the deque lines");

constexpr uint32_t kMaxBlockThreads = 256;
// Free small-frame stack per workgroup: two depot chunks (FMM tasks take
// frames only when exposed to thieves; a smaller stack leaves room for a
// sixth workgroup per CU)
constexpr uint32_t kBlockStackSmall = 2 * kChunkSmall;
constexpr uint32_t kP2PTile = 64;
constexpr uint32_t kBlkLocal = 128;  // private stack of cell-pair task images
constexpr uint32_t kM2LSlots = 1024; // >= ceil(924 / threads) * threads for 64, 128, 256 threads

struct BlockLds {
  uint32_t stk_s[kBlockStackSmall];
  uint32_t stk_b[kStackBig];
  uint32_t fw[kFrameWords];     // frame of the current task
  uint32_t task, next, next_cont, stop;
  uint32_t out_type, nchild, ckind, pad0;
  int64_t value;
  uint32_t child[8][2];         // FMM: children to fork (A, B)
  // FMM batch: the cell records of the task's pair (rec 0 = A, rec 1 = B) and
  // of the cells a split created (rec 2 + c); pair i of the batch is
  // (pid[i][0], pid[i][1]) with records (prec[i][0], prec[i][1])
  int32_t rec[10][fmm::kCellInts];
  uint32_t pid[8][2];
  uint8_t prec[8][2];
  uint32_t n_m2l, n_p2p, m2l_idx[8], p2p_idx[8];
  // P2P batch: target point ranges x source point ranges (one side is one cell)
  int32_t tr_b[8], tr_n[8], sr_b[8], sr_n[8];
  uint32_t nt, ns;
  uint32_t first_fail;          // UTS: first failed draw in a batch
  int64_t bottom, top_seen;     // owner's view of its deque
  union {                       // the M2L batch completes before the P2P batch starts
    double Tc[8][fmm::kNc];     // Taylor coefficients of the batch's M2L pairs
    double red[kMaxBlockThreads];  // P2P: partial sums of the source groups
    double pstage[8 * fmm::kNc];   // P2P: [kMaxBlockThreads, +256) staged source chunks
  };
  double QBc[8][fmm::kNc];      // source moments of the M2L pairs
  double dl[8][4];              // M2L pair i: centre difference A - B and the reciprocal of its squared length
  uint32_t dmt[fmm::kNc][2];    // Taylor recursion indices of coefficient t: g - e_c (byte c of [0]), g - 2 e_c ([1])
  uint4 lstk[2 * kBlkLocal];    // private stack (frame words 0..7 of each task)
  uint32_t lbot, ltop, local, dry;
  // M2L term table, copied once per workgroup:
  // a | b << 8 | (a+b) << 16 | coefficient << 24 (the coefficient
  // C(a+b, a) (-1)^|b| is an integer of magnitude <= 20, kept as int8).
  // Thread t owns the consecutive terms [t*C, (t+1)*C) (C = ceil(924 /
  // threads)); its r-th term is stored at r * threads + t so that a round of
  // loads touches consecutive words.
  uint32_t mab[kM2LSlots];
  // Running sums for the target cell of consecutive pairs (siblings of one
  // split share it): M2L local coefficients of cell lcell, P2P potentials of
  // the points of leaf pcell.  Added to memory when the target changes.
  double lacc[fmm::kNc];
  double pacc[kP2PTile];
  const fmm::FmmDesc *ldesc;
  const fmm::FmmDesc *pdesc;
  uint32_t lcell, pcell;
  int32_t pbegin, pn;
};

// Add the running M2L / P2P sums of the workgroup to memory (all threads).
template <int NT>
GTAP_DEV void fmm_flush_acc(BlockLds &S, bool m2l, bool p2p) {
  const uint32_t tx = threadIdx.x;
  if (m2l && S.lcell != kNone) {
    for (uint32_t t = tx; t < static_cast<uint32_t>(fmm::kNc); t += NT) {
      unsafeAtomicAdd(S.ldesc->L + static_cast<size_t>(S.lcell) * fmm::kNc + t, S.lacc[t]);
      S.lacc[t] = 0.0;
    }
  }
  if (p2p && S.pcell != kNone) {
    for (uint32_t t = tx; t < static_cast<uint32_t>(S.pn); t += NT) {
      unsafeAtomicAdd(S.pdesc->phi + S.pbegin + t, S.pacc[t]);
      S.pacc[t] = 0.0;
    }
  }
  __syncthreads();
  if (tx == 0) {
    if (m2l) S.lcell = kNone;
    if (p2p) S.pcell = kNone;
  }
  __syncthreads();
}

GTAP_DEV ClDeque *cl_deque(const Params &p, uint32_t w) { return reinterpret_cast<ClDeque *>(p.dq) + w; }
GTAP_DEV uint32_t *cl_buf(const Params &p, uint32_t w) { return p.rings + static_cast<size_t>(w) * p.cap; }

// Owner pop (thread 0).  Returns kNone when the deque is empty.
GTAP_DEV uint32_t cl_pop(const Params &p, BlockLds &S, uint32_t me) {
  const int64_t b = S.bottom - 1;
  if (b < S.top_seen) return kNone;  // top only grows: certainly empty
  ClDeque *d = cl_deque(p, me);
  __hip_atomic_exchange(&d->bottom, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  drain();
  int64_t t = static_cast<int64_t>(co_ld64(reinterpret_cast<const uint64_t *>(&d->top)));
  S.top_seen = t;
  if (t > b) {
    co_st64(reinterpret_cast<uint64_t *>(&d->bottom), static_cast<uint64_t>(b + 1));
    return kNone;
  }
  const uint32_t x = co_ld32(cl_buf(p, me) + (static_cast<uint64_t>(b) & (p.cap - 1)));
  if (t == b) {
    int64_t e = t;
    const bool won = cas_relaxed(&d->top, &e, t + 1);
    co_st64(reinterpret_cast<uint64_t *>(&d->bottom), static_cast<uint64_t>(b + 1));
    S.top_seen = t + 1;
    return won ? x : kNone;
  }
  S.bottom = b;
  return x;
}

// Thief (thread 0): one task from the top of worker v's deque, or kNone.
GTAP_DEV uint32_t cl_steal(const Params &p, uint32_t v) {
  ClDeque *d = cl_deque(p, v);
  int64_t t = static_cast<int64_t>(co_ld64(reinterpret_cast<const uint64_t *>(&d->top)));
  drain();
  const int64_t b = static_cast<int64_t>(co_ld64(reinterpret_cast<const uint64_t *>(&d->bottom)));
  drain();
  if (t >= b) return kNone;
  const uint32_t x = co_ld32(cl_buf(p, v) + (static_cast<uint64_t>(t) & (p.cap - 1)));
  drain();
  int64_t e = t;
  return cas_relaxed(&d->top, &e, t + 1) ? x : kNone;
}

// Publish n IDs (already written to the slots by wavefront 0) at the bottom.
GTAP_DEV bool cl_room(const Params &p, BlockLds &S, uint32_t me, uint32_t n) {
  if (S.bottom + n - S.top_seen <= static_cast<int64_t>(p.cap)) return true;
  S.top_seen = static_cast<int64_t>(co_ld64(reinterpret_cast<const uint64_t *>(&cl_deque(p, me)->top)));
  return S.bottom + n - S.top_seen <= static_cast<int64_t>(p.cap);
}

GTAP_DEV void store_result(const Params &p, uint32_t job, int64_t v) {
  JobSlot &J = p.jobs[job];
  st_relaxed(&J.result, v);
  st_relaxed(&J.t_done, wall_ticks());
  st_relaxed(&J.done, 1u);
}

// ---- FMM cell-pair body (all threads) -------------------------------------------
// Statistics of the FMM job a workgroup works on, flushed when the job changes.
struct FmmCounters {
  uint32_t job;
  uint64_t m2l, p2p, m2l_hash, p2p_hash, inter;
  const fmm::FmmDesc *desc;  // descriptor of `job` (read once per job)
  int64_t ta, tb;            // its MAC parameter theta = ta / tb
};

GTAP_DEV void fmm_flush(const Params &p, FmmCounters &fc) {
  if (fc.job == kNone) return;
  if (threadIdx.x == 0) {
    fmm::FmmDesc *D = reinterpret_cast<fmm::FmmDesc *>(co_ld64(&p.jobs[fc.job].a[0]));
    if (fc.m2l) fetch_add_relaxed(&D->m2l_pairs, fc.m2l);
    if (fc.p2p) fetch_add_relaxed(&D->p2p_pairs, fc.p2p);
    if (fc.m2l_hash) fetch_add_relaxed(&D->m2l_hash, fc.m2l_hash);
    if (fc.p2p_hash) fetch_add_relaxed(&D->p2p_hash, fc.p2p_hash);
    if (fc.inter) fetch_add_relaxed(&D->p2p_inter, fc.inter);
  }
  fc = FmmCounters{kNone, 0, 0, 0, 0, 0, nullptr, 0, 1};
}

// Lane k's value of x (k wave-uniform), read through two 32-bit lane reads.
GTAP_DEV double lane_double(double x, int32_t k) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(b)), k));
  const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(b >> 32)), k));
  return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

constexpr bool m2l_coefficients_fit_int8() {
  const fmm::Tables T = fmm::make_tables();
  for (int m = 0; m < fmm::kM2LTerms; ++m) {
    const double c = T.m2l_c[m];
    if (c != static_cast<double>(static_cast<int32_t>(c)) || c > 127.0 || c < -127.0) return false;
  }
  return true;
}
static_assert(m2l_coefficients_fit_int8(), "the M2L term table packs its coefficients as int8");

// Branch of the pair of cell records (A, B): 1 accept (M2L), 2 both leaves
// (P2P), 0 split.
GTAP_DEV uint32_t fmm_branch(const int32_t *A, const int32_t *B, const FmmCounters &fc) {
  if (fmm::mac_accept(A, B, fc.ta, fc.tb)) return 1;
  return (A[7] == 0 && B[7] == 0) ? 2u : 0u;
}

// Make cell `a` the target of the workgroup's running sums (M2L: local
// coefficients, P2P: potentials of its points), adding the previous target's
// sums to memory first.  All threads; every thread reads the same state
// because the last change was followed by a barrier (the callers end their
// pass with one, which also orders thread 0's update of the target before
// the next check).
template <int NT>
GTAP_DEV void fmm_target(BlockLds &S, const fmm::FmmDesc *D, uint32_t a, bool m2l, int32_t pbegin = 0,
                         int32_t pn = 0) {
  const bool same = m2l ? (S.lcell == a && S.ldesc == D) : (S.pcell == a && S.pdesc == D);
  if (same) return;
  const uint32_t tx = threadIdx.x;
  if (m2l) {
    if (S.lcell != kNone) {
      for (uint32_t t = tx; t < static_cast<uint32_t>(fmm::kNc); t += NT) {
        unsafeAtomicAdd(S.ldesc->L + static_cast<size_t>(S.lcell) * fmm::kNc + t, S.lacc[t]);
        S.lacc[t] = 0.0;
      }
    }
  } else if (S.pcell != kNone) {
    for (uint32_t t = tx; t < static_cast<uint32_t>(S.pn); t += NT) {
      unsafeAtomicAdd(S.pdesc->phi + S.pbegin + t, S.pacc[t]);
      S.pacc[t] = 0.0;
    }
  }
  __syncthreads();  // every thread has read the old target and cleared its sums
  if (tx == 0) {
    if (m2l) {
      S.lcell = a;
      S.ldesc = D;
    } else {
      S.pcell = a;
      S.pdesc = D;
      S.pbegin = pbegin;
      S.pn = pn;
    }
  }
}

// M2L(A <- B) for the batch's pairs m2l_idx[0 .. n): Taylor coefficients of
// 1/|d + h| degree by degree for all of them at once, then each pair's 924
// terms spread evenly over the workgroup into the running sums of its target.
constexpr double kInvDeg[fmm::kP + 1] = {0.0, 1.0, 1.0 / 2, 1.0 / 3, 1.0 / 4, 1.0 / 5, 1.0 / 6};
static_assert(fmm::kP == 6, "reciprocal table of the Taylor degrees");

template <int NT>
GTAP_DEV void fmm_m2l_batch(const Params &p, BlockLds &S, const fmm::FmmDesc *D, FmmCounters &fc) {
  const uint32_t tx = threadIdx.x;
  const uint32_t n = S.n_m2l;
  if (n == 0) return;
  auto delta = [&](uint32_t i, double &d0, double &d1, double &d2) {
    const uint32_t k = S.m2l_idx[i];
    const int32_t *A = S.rec[S.prec[k][0]], *B = S.rec[S.prec[k][1]];
    d0 = fmm::cell_centre(A[1], A[0]) - fmm::cell_centre(B[1], B[0]);
    d1 = fmm::cell_centre(A[2], A[0]) - fmm::cell_centre(B[2], B[0]);
    d2 = fmm::cell_centre(A[3], A[0]) - fmm::cell_centre(B[3], B[0]);
  };
  // source moments of every pair (one round of loads), and T_0
  for (uint32_t x = tx; x < n * static_cast<uint32_t>(fmm::kNc); x += NT) {
    const uint32_t i = x / fmm::kNc, t = x - i * fmm::kNc;
    S.QBc[i][t] = D->Q[static_cast<size_t>(S.pid[S.m2l_idx[i]][1]) * fmm::kNc + t];
  }
  if (tx < n) {
    double d0, d1, d2;
    delta(tx, d0, d1, d2);
    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    S.dl[tx][0] = d0;
    S.dl[tx][1] = d1;
    S.dl[tx][2] = d2;
    S.dl[tx][3] = 1.0 / r2;
    S.Tc[tx][0] = 1.0 / sqrt(r2);
  }
  __syncthreads();
  // Degree by degree; wavefront w takes the pairs w, w + G, ..., so every
  // coefficient a lane reads was written by its own wavefront in an earlier
  // degree (LDS accesses of one wavefront complete in order): one barrier
  // after the last degree instead of one per degree.
  {
    constexpr uint32_t G = NT / kWave;
    const uint32_t wv = tx / kWave, ln = tx % kWave;
    const uint32_t nw = n > wv ? (n - wv + G - 1) / G : 0u;
    for (int deg = 1; deg <= fmm::kP; ++deg) {
      const uint32_t lo = static_cast<uint32_t>(fmm::ncoef(deg - 1)), nd = static_cast<uint32_t>(fmm::ncoef(deg)) - lo;
      for (uint32_t x = ln; x < nw * nd; x += kWave) {
        const uint32_t ii = x / nd, t = lo + (x - ii * nd);
        const uint32_t i = wv + ii * G;
        const uint32_t m1w = S.dmt[t][0], m2w = S.dmt[t][1];
        double s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const uint32_t m1 = (m1w >> (8 * c)) & 0xFFu, m2 = (m2w >> (8 * c)) & 0xFFu;
          if (m1 != 0xFFu) s1 += S.dl[i][c] * S.Tc[i][m1];
          if (m2 != 0xFFu) s2 += S.Tc[i][m2];
        }
        S.Tc[i][t] = -((2.0 * deg - 1.0) * s1 + (deg - 1.0) * s2) * (S.dl[i][3] * kInvDeg[deg]);
      }
      wave_sync();
    }
  }
  __syncthreads();
  // Consecutive pairs with the same target (all of them when the split took
  // the source side) share one pass over the terms: each term adds its
  // coefficient times the sum over those pairs.
  constexpr uint32_t C = (fmm::kM2LTerms + NT - 1) / NT;
  for (uint32_t i = 0; i < n;) {
    const uint32_t a = S.pid[S.m2l_idx[i]][0];
    uint32_t j = i + 1;
    while (j < n && S.pid[S.m2l_idx[j]][0] == a) ++j;
    fmm_target<NT>(S, D, a, true);
    uint32_t cur = 0xFFu;
    double acc = 0.0;
#pragma unroll
    for (uint32_t r = 0; r < C; ++r) {
      const uint32_t w = S.mab[r * NT + tx];
      const uint32_t at = w & 0xFFu;
      if (at != cur) {
        if (cur != 0xFFu) atomicAdd(&S.lacc[cur], acc);
        acc = 0.0;
        cur = at;
      }
      if (at != 0xFFu) {
        const uint32_t g = (w >> 16) & 0xFFu, bq = (w >> 8) & 0xFFu;
        double sum = 0.0;
        for (uint32_t q = i; q < j; ++q) sum += S.Tc[q][g] * S.QBc[q][bq];
        acc += static_cast<double>(static_cast<int8_t>(w >> 24)) * sum;
      }
    }
    if (cur != 0xFFu) atomicAdd(&S.lacc[cur], acc);
    for (uint32_t q = i; q < j; ++q) {
      fc.m2l += 1;
      fc.m2l_hash += fmm::pair_hash(a, S.pid[S.m2l_idx[q]][1]);
    }
    __syncthreads();  // the sums are complete before a change of target adds them to memory
    i = j;
  }
}

// P2P for the batch's leaf pairs p2p_idx[0 .. n).  They share one cell --
// the target if the split took the source side, the source otherwise -- so
// the batch is (target ranges) x (source ranges) and runs as one pass:
// target = tx mod 64 over the concatenated target ranges; wavefront w takes
// the chunks w, w + G, ... of 64 / G concatenated sources (G wavefronts),
// loads a chunk with one coalesced load per lane and walks it by reading each
// source from its lane (one round of loads per chunk, no LDS staging, no
// barriers in the source loop).
template <int NT>
GTAP_DEV void fmm_p2p_batch(BlockLds &S, const fmm::FmmDesc *D, FmmCounters &fc) {
  const uint32_t tx = threadIdx.x;
  const uint32_t n = S.n_p2p;
  if (n == 0) return;
  if (tx < kWave) {
    // ranges, pair q on lane q of wavefront 0: the shared cell once (from the
    // first pair), the other side per pair, compacted in pair order
    const bool act = tx < n;
    const int32_t *A = S.rec[0], *B = S.rec[0];
    bool ft = false, fs = false;
    uint64_t h = 0, in = 0;
    if (act) {
      const uint32_t k = S.p2p_idx[tx], k0 = S.p2p_idx[0];
      A = S.rec[S.prec[k][0]];
      B = S.rec[S.prec[k][1]];
      const uint32_t a = S.pid[k][0], b = S.pid[k][1];
      ft = tx == 0 || S.prec[k][0] != S.prec[k0][0];
      fs = tx == 0 || S.prec[k][1] != S.prec[k0][1];
      const int64_t na = A[5] - A[4], nb = B[5] - B[4];
      h = fmm::pair_hash(a, b);
      in = static_cast<uint64_t>(na * nb - (a == b ? na : 0));
    }
    const uint64_t mt = ballot(ft), ms = ballot(fs);
    if (ft) {
      const uint32_t r = rank_below(mt);
      S.tr_b[r] = A[4];
      S.tr_n[r] = A[5] - A[4];
    }
    if (fs) {
      const uint32_t r = rank_below(ms);
      S.sr_b[r] = B[4];
      S.sr_n[r] = B[5] - B[4];
    }
    const uint64_t hs = wave_inclusive_sum64(h), is = wave_inclusive_sum64(in);
    const uint64_t hsum = readlane64(hs, 63), isum = readlane64(is, 63);
    if (tx == 0) {
      // thread 0 keeps the job's statistics
      fc.p2p += n;
      fc.p2p_hash += hsum;
      fc.inter += isum;
      S.nt = __popcll(mt);
      S.ns = __popcll(ms);
    }
  }
  __syncthreads();
  constexpr uint32_t G = NT / kP2PTile;
  const int32_t wsrc = static_cast<int32_t>(__builtin_amdgcn_readfirstlane(tx / kP2PTile));
  const uint32_t nt = S.nt, ns = S.ns;
  const uint32_t ln = tx & (kWave - 1);
  int32_t total = 0, stotal = 0;
  for (uint32_t r = 0; r < nt; ++r) total += S.tr_n[r];
  for (uint32_t r = 0; r < ns; ++r) stotal += S.sr_n[r];
  // one target cell of at most 64 points: its sums stay in LDS across tasks
  const bool keep_sum = nt == 1 && total <= static_cast<int32_t>(kP2PTile);
  if (keep_sum) fmm_target<NT>(S, D, S.pid[S.p2p_idx[0]][0], false, S.tr_b[0], total);
  uint32_t coinc = 0;
  const double *__restrict__ px = D->px, *__restrict__ py = D->py, *__restrict__ pz = D->pz,
               *__restrict__ pq = D->pq;
  for (int32_t t0 = 0; t0 < total; t0 += kP2PTile) {
    const int32_t g = t0 + static_cast<int32_t>(tx % kP2PTile);
    const bool live = g < total;
    int32_t i = 0;
    if (live) {  // the g-th point of the concatenated target ranges
      int32_t off = g;
      uint32_t r = 0;
      while (off >= S.tr_n[r]) {
        off -= S.tr_n[r];
        ++r;
      }
      i = S.tr_b[r] + off;
    }
    double xi = 0.0, yi = 0.0, zi = 0.0;
    if (live) {
      xi = px[i];
      yi = py[i];
      zi = pz[i];
    }
    double acc = 0.0;
    // chunks of SC = 64 / G sources, so that a batch of up to 64 sources
    // still keeps every wavefront busy
    constexpr int32_t SC = static_cast<int32_t>(kWave / G);
    // each wavefront's chunk, staged in LDS behind the reduction slots (the
    // M2L coefficients' space, free during P2P) and read back by all lanes
    // from one address per source
    static_assert(kMaxBlockThreads + kWave * 4 <= 8 * fmm::kNc, "P2P staging space");
    double *const stage = S.pstage + kMaxBlockThreads + static_cast<uint32_t>(wsrc) * static_cast<uint32_t>(SC) * 4u;
    for (int32_t c0 = wsrc * SC; c0 < stotal; c0 += static_cast<int32_t>(G) * SC) {
      // this lane's source of the chunk: the (c0 + lane)-th of the concatenated ranges
      int32_t sj = -1;
      double sx = 0.0, sy = 0.0, sz = 0.0, sq = 0.0;
      int32_t off = c0 + static_cast<int32_t>(ln);
      if (static_cast<int32_t>(ln) < SC && off < stotal) {
        uint32_t r = 0;
        while (off >= S.sr_n[r]) {
          off -= S.sr_n[r];
          ++r;
        }
        sj = S.sr_b[r] + off;
        sx = px[sj];
        sy = py[sj];
        sz = pz[sj];
        sq = pq[sj];
      }
      if (static_cast<int32_t>(ln) < SC) {
        reinterpret_cast<double2 *>(stage)[2 * ln] = make_double2(sx, sy);
        reinterpret_cast<double2 *>(stage)[2 * ln + 1] = make_double2(sz, sq);
      }
      wave_sync();
      const int32_t nk = (stotal - c0) < SC ? (stotal - c0) : SC;
      for (int32_t k = 0; k < nk; ++k) {
        const double2 s0 = reinterpret_cast<const double2 *>(stage)[2 * k];
        const double2 s1 = reinterpret_cast<const double2 *>(stage)[2 * k + 1];
        const double dx = xi - s0.x, dy = yi - s0.y, dz = zi - s1.x;
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 == 0.0) {
          if (live && __builtin_amdgcn_readlane(sj, k) != i) ++coinc;
        } else {
          acc += s1.y * fmm::rsqrt_nr(r2);
        }
      }
      wave_sync();  // the chunk's reads are issued before the next chunk overwrites it
    }
    __syncthreads();
    S.red[tx] = acc;
    __syncthreads();
    if (tx < kP2PTile && live) {
      double sum = 0.0;
#pragma unroll
      for (uint32_t q = 0; q < G; ++q) sum += S.red[tx + q * kP2PTile];
      if (keep_sum) S.pacc[tx] += sum;
      else unsafeAtomicAdd(D->phi + i, sum);
    }
  }
  if (coinc) atomicAdd(reinterpret_cast<unsigned long long *>(const_cast<uint64_t *>(&D->coincident)),
                       static_cast<unsigned long long>(coinc));
  __syncthreads();  // S.red and the ranges are free for the next pass
}

// One cell-pair task (A, B) of the dual-tree traversal.  An accepted pair
// runs M2L, a pair of leaves P2P.  Otherwise the wider cell splits, and the
// workgroup classifies all the child pairs at once: accepted children run
// their M2L together and leaf pairs their P2P inside this task; only
// children that must split again become tasks (S.child, S.nchild).  The
// traversal visits the same pairs as one task per pair would.
template <int NT>
GTAP_DEV void fmm_pair(const Params &p, BlockLds &S, uint32_t job, FmmCounters &fc) {
  const uint32_t tx = threadIdx.x;
  const uint32_t a = S.fw[FW_P0], b = S.fw[FW_P0 + 1];
  if (fc.job != job) {
    fmm_flush(p, fc);
    fc.job = job;
    fc.desc = reinterpret_cast<const fmm::FmmDesc *>(co_ld64(&p.jobs[job].a[0]));
    fc.ta = fc.desc->ta;
    fc.tb = fc.desc->tb;
  }
  const fmm::FmmDesc *D = fc.desc;
  if (tx < fmm::kCellInts) {
    S.rec[0][tx] = D->cell[static_cast<size_t>(a) * fmm::kCellInts + tx];
    S.rec[1][tx] = D->cell[static_cast<size_t>(b) * fmm::kCellInts + tx];
  }
  __syncthreads();
  // Every thread decides the pair's branch and, for a split, which cell
  // splits, from the records in LDS (the same values): the children's
  // records are loaded right away, with no round through thread 0.
  const int32_t *A = S.rec[0], *B = S.rec[1];
  const uint32_t br0 = fmm_branch(A, B, fc);
  uint32_t k = 0, first = 0;
  bool split_a = false;
  if (br0 == 0) {
    // split the wider cell; on a tie the target unless it is a leaf; never a leaf
    split_a = A[0] < B[0] ? true : (A[0] > B[0] ? false : A[7] != 0);
    if (split_a && A[7] == 0) split_a = false;
    if (!split_a && B[7] == 0) split_a = true;
    const int32_t *Sp = split_a ? A : B;
    k = static_cast<uint32_t>(Sp[7]);
    first = static_cast<uint32_t>(Sp[6]);
  }
  if (k == 0) {
    if (tx == 0) {
      S.n_m2l = br0 == 1 ? 1u : 0u;
      S.n_p2p = br0 == 2 ? 1u : 0u;
      S.pid[0][0] = a;
      S.pid[0][1] = b;
      S.prec[0][0] = 0;
      S.prec[0][1] = 1;
      S.m2l_idx[0] = 0;
      S.p2p_idx[0] = 0;
      S.nchild = 0;
    }
    __syncthreads();
  } else {
    // the new cells' records (one round of loads), then every child's branch
    if (tx < k * fmm::kCellInts) {
      const uint32_t c = tx / fmm::kCellInts, w = tx - c * fmm::kCellInts;
      S.rec[2 + c][w] = D->cell[static_cast<size_t>(first + c) * fmm::kCellInts + w];
    }
    __syncthreads();
    // child c on lane c of wavefront 0: its pair and records, its branch;
    // ballots compact the M2L, P2P and split-again lists in child order
    if (tx < kWave) {
      const bool act = tx < k;
      uint32_t br = 3u, p0 = 0, p1 = 0;
      if (act) {
        const uint32_t ch = first + tx;
        p0 = split_a ? ch : a;
        p1 = split_a ? b : ch;
        const uint32_t r0 = split_a ? 2 + tx : 0u, r1 = split_a ? 1u : 2 + tx;
        S.pid[tx][0] = p0;
        S.pid[tx][1] = p1;
        S.prec[tx][0] = static_cast<uint8_t>(r0);
        S.prec[tx][1] = static_cast<uint8_t>(r1);
        br = fmm_branch(S.rec[r0], S.rec[r1], fc);
      }
      const uint64_t mm = ballot(br == 1), mp = ballot(br == 2), mf = ballot(br == 0);
      if (br == 1) {
        S.m2l_idx[rank_below(mm)] = tx;
      } else if (br == 2) {
        S.p2p_idx[rank_below(mp)] = tx;
      } else if (br == 0) {
        const uint32_t f = rank_below(mf);
        S.child[f][0] = p0;
        S.child[f][1] = p1;
      }
      if (tx == 0) {
        S.n_m2l = __popcll(mm);
        S.n_p2p = __popcll(mp);
        S.nchild = __popcll(mf);
      }
    }
    __syncthreads();
  }
  fmm_m2l_batch<NT>(p, S, D, fc);
  fmm_p2p_batch<NT>(S, D, fc);
}

// Root frame of job j in block mode.
GTAP_DEV void write_root_block(const Params &p, uint32_t id, uint32_t j) {
  const uint32_t jkind = static_cast<uint32_t>(co_ld64(reinterpret_cast<const uint64_t *>(p.jobs + j)));
  if (jkind == 5) {  // FMM: the (root, root) cell pair
    ChildInit c{};
    write_frame(frame_ptr(p, id), kNone, j, state_word(TK_FMM, 0, 0), c);
  } else {
    write_root(p, id, j);
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void block_sched_kernel(Params p) {
  static_assert(NT % kWave == 0 && NT <= static_cast<int>(kMaxBlockThreads), "workgroup shape");
  __shared__ BlockLds S;
  const uint32_t tx = threadIdx.x, ln = tx & 63u, wv = tx >> 6;
  const uint32_t me = blockIdx.x;
  const uint32_t nw = gridDim.x;
  const uint64_t deadline = wall_ticks() + p.timeout_ticks;
  PoolView PS{S.stk_s, 0, 0, 0, kBlockStackSmall, kChunkSmall, p.bins_s, p.store_s,
              p.bincap_s, &p.ctl->bump_small, p.nframes_s, 0u, 0};
  PoolView PB{S.stk_b, 0, 0, 0, kStackBig, kChunkBig, p.bins_b, p.store_b,
              p.bincap_b, &p.ctl->bump_big, p.nframes_b, kBigBit, 1};
  WaveCounters wc;
  for (int i = 0; i < static_cast<int>(ST_COUNT); ++i) wc.v[i] = 0;
  FmmCounters fc{kNone, 0, 0, 0, 0, 0, nullptr, 0, 1};
  uint32_t rng = 0x9E3779B9u ^ (me * 0x85EBCA6Bu + 1u);
  uint64_t t_loop = clock64(), busy_cycles = 0, idle_cycles = 0;
  if (tx == 0) {
    S.bottom = 0;
    S.top_seen = 0;
    S.stop = 0;
    S.lbot = 0;
    S.ltop = 0;
    S.local = 0;
    S.dry = 0;
  }
  {
    constexpr uint32_t C = (fmm::kM2LTerms + NT - 1) / NT;
    static_assert(C * NT <= kM2LSlots, "M2L term slots");
    for (uint32_t r = 0; r < C; ++r) {
      const uint32_t m = tx * C + r;  // this thread's r-th term
      uint32_t w = 0xFFu;
      if (m < static_cast<uint32_t>(fmm::kM2LTerms)) {
        uint32_t at = 0;
        while (fmm::kTab.m2l_first[at + 1] <= m) ++at;
        const int32_t c = static_cast<int32_t>(fmm::kTab.m2l_c[m]);
        w = at | (static_cast<uint32_t>(fmm::kTab.m2l_b[m]) << 8) | (static_cast<uint32_t>(fmm::kTab.m2l_g[m]) << 16) |
            (static_cast<uint32_t>(static_cast<uint8_t>(static_cast<int8_t>(c))) << 24);
      }
      S.mab[r * NT + tx] = w;
    }
  }
  for (uint32_t t = tx; t < static_cast<uint32_t>(fmm::kNc); t += NT) {
    S.lacc[t] = 0.0;
    S.dmt[t][0] = fmm::kTab.dm1[t][0] | (fmm::kTab.dm1[t][1] << 8) | (fmm::kTab.dm1[t][2] << 16);
    S.dmt[t][1] = fmm::kTab.dm2[t][0] | (fmm::kTab.dm2[t][1] << 8) | (fmm::kTab.dm2[t][2] << 16);
  }
  for (uint32_t t = tx; t < kP2PTile; t += NT) S.pacc[t] = 0.0;
  if (tx == 0) {
    S.lcell = kNone;
    S.pcell = kNone;
    S.ldesc = nullptr;
    S.pdesc = nullptr;
    S.pbegin = 0;
    S.pn = 0;
  }
  __syncthreads();
  // counted cell-pair tasks (thread 0's registers): the job they belong to
  // and its unadded outstanding-count delta
  uint32_t cjob = kNone;
  int64_t cdelta = 0;
  auto cflush = [&](bool positive_only) {
    if (cjob == kNone || cdelta == 0 || (positive_only && cdelta < 0)) return;
    int64_t *pc = &p.jobs[cjob].pending;
    if (cdelta > 0) {
      fetch_add_relaxed(pc, cdelta);  // cannot end the job: no wait
    } else {
      const int64_t old = fetch_add_relaxed(pc, cdelta);
      if (old + cdelta == 0) {  // the job's last task completed here
        store_result(p, cjob, 0);
        drain();
        fetch_add_relaxed(&p.ctl->jobs_remaining, -1);
      }
    }
    cdelta = 0;
  };

  // roots: job j goes to worker j mod nw, onto its deque
  if (wv == 0) {
    const uint32_t nroots = me < p.njobs ? (p.njobs - me + nw - 1) / nw : 0u;
    AllocResult ar{};
    if (nroots > p.cap) {
      if (ln == 0) raise_error(p, -6 /*GTAP_E_CAPACITY*/, 2, p.cap, nroots, me, -1);
    } else if (nroots > 0 && alloc_frames(p, PS, me, nroots, ar, wc)) {
      wave_sync();
      for (uint32_t g = ln; g < nroots; g += kWave) {
        const uint32_t id = alloc_id(PS, ar, g);
        write_root_block(p, id, me + g * nw);
        co_st32(cl_buf(p, me) + g, id);
      }
      drain();
      if (ln == 0) {
        co_st64(reinterpret_cast<uint64_t *>(&cl_deque(p, me)->bottom), nroots);
        S.bottom = nroots;
      }
    }
  }
  __syncthreads();

  uint32_t tid = kNone, cont = 0, idle = 0, iter = 0;
  for (;;) {
    // ---- acquire: own deque, then random victims ----
    if (tid == kNone) {
      if (tx == 0) {
        uint32_t t = kNone;
        S.local = 0;
        if (S.ltop != S.lbot) {
          // private stack, newest first: the image becomes the frame copy
          const uint32_t e = (S.ltop - 1) & (kBlkLocal - 1);
          const uint4 a = S.lstk[2 * e], b = S.lstk[2 * e + 1];
          S.fw[0] = a.x; S.fw[1] = a.y; S.fw[2] = a.z; S.fw[3] = a.w;
          S.fw[4] = b.x; S.fw[5] = b.y; S.fw[6] = b.z; S.fw[7] = b.w;
          S.ltop -= 1;
          S.local = 1;
        } else {
          t = cl_pop(p, S, me);
        }
        if (t != kNone) {
          wc.add(ST_POPPED, 1);
        } else if (S.local) {
        } else if (nw > 1) {
          wc.add(ST_STEAL_ATTEMPTS, 1);
          for (uint32_t k = 0; k < p.steal_probes && t == kNone; ++k) {
            uint32_t v = xorshift32(rng) % (nw - 1);
            if (v >= me) ++v;
            t = cl_steal(p, v);
          }
          if (t != kNone) wc.add(ST_STOLEN, 1);
        }
        S.task = t;
        S.next_cont = 0;
        uint32_t stop = 0;
        if (t == kNone && !S.local) cflush(false);  // nothing to run: report completions
        if (t == kNone && !S.local && (idle & 3u) == 0u) {
          if (ld_relaxed(&p.ctl->jobs_remaining) <= 0 || ld_relaxed(&p.ctl->error) != 0) stop = 1;
          else if (wall_ticks() > deadline) {
            raise_error(p, -8 /*GTAP_E_TIMEOUT*/, 3, p.timeout_ticks, 0, me, -1);
            stop = 1;
          }
        }
        S.stop = stop;
      }
      __syncthreads();
      tid = S.task;
      cont = 0;
      if (S.stop) break;
      if (tid == kNone && !S.local) {
        ++idle;
        wc.add(ST_IDLE, 1);
        backoff_sleep(idle);
        const uint64_t now = clock64();
        idle_cycles += now - t_loop;
        t_loop = now;
        __syncthreads();
        continue;
      }
    }
    idle = 0;
    ++iter;
    wc.add(ST_ITERS, 1);
    if ((iter & 63u) == 0) {
      if (tx == 0) {
        uint32_t stop = 0;
        if (ld_relaxed(&p.ctl->error) != 0) stop = 1;
        else if (wall_ticks() > deadline) {
          raise_error(p, -8 /*GTAP_E_TIMEOUT*/, 3, p.timeout_ticks, 0, me, -1);
          stop = 1;
        }
        S.stop = stop;
      }
      __syncthreads();
      if (S.stop) break;
    }

    // ---- load the frame (a private-stack image is already in place) ----
    const bool from_local = (tid == kNone);
    if (!from_local && tx < kFrameWords) S.fw[tx] = co_ld32(frame_ptr(p, tid) + tx);
    if (tx == 0) {
      S.out_type = OUT_DONE;
      S.nchild = 0;
      S.value = 0;
    }
    __syncthreads();
    const uint32_t kind = S.fw[FW_STATE] & 0xFFu;
    const uint32_t job = S.fw[FW_JOB];
    if (cont) wc.add(ST_CONTS, 1);
    else wc.add(ST_TASKS, 1);

    // ---- body ----
    if (cont) {
      if (tx == 0) {
        const int64_t jw = static_cast<int64_t>(pack(S.fw[FW_JOIN], S.fw[FW_JOIN + 1]));
        const int64_t big = static_cast<int64_t>(pack(S.fw[FW_BIGACC], S.fw[FW_BIGACC + 1]));
        S.value = (jw >> kJoinBits) + big + (kind == TK_UTS ? 1 : 0);
      }
    } else if (kind == TK_FIB) {
      if (tx == 0) {
        const uint32_t n = S.fw[FW_P0];
        if (n < 2) {
          S.value = n;
        } else {
          S.out_type = OUT_FORK;
          S.nchild = 2;
        }
      }
    } else if (kind == TK_UTS) {
      // cooperative geometric draw: the child count is the index of the first
      // failed draw j = 1, 2, ...
      const uint64_t id = pack(S.fw[FW_P0], S.fw[FW_P0 + 1]);
      const uint32_t dm = S.fw[FW_P0 + 2];
      const uint64_t thr = pack(S.fw[FW_P0 + 3], S.fw[FW_P0 + 4]);
      if ((dm & 0xFFFFu) < (dm >> 16)) {
        uint32_t base = 0;
        for (;;) {
          if (tx == 0) S.first_fail = kNone;
          __syncthreads();
          const uint64_t j = base + tx + 1;
          if (!(mix64(id ^ (j * 0xD1B54A32D192ED03ull)) < thr)) atomicMin(&S.first_fail, base + tx);
          __syncthreads();
          const uint32_t ff = S.first_fail;
          __syncthreads();
          if (ff != kNone) {
            if (tx == 0 && ff > 0) {
              S.out_type = OUT_FORK;
              S.nchild = ff;
            }
            break;
          }
          base += NT;
        }
      }
      if (tx == 0 && S.out_type == OUT_DONE) S.value = 1;
    } else if (kind == TK_FMM) {
      fmm_pair<NT>(p, S, job, fc);
      if (tx == 0 && S.nchild > 0) S.out_type = OUT_FORK;  // the pairs that split again
    }
    __syncthreads();

    // ---- fork or complete (wavefront 0) ----
    if (wv == 0 && kind == TK_FMM) {
      // counted cell-pair task: children onto the private stack, completion
      // into the job's outstanding count
      const uint32_t k = (S.out_type == OUT_FORK) ? S.nchild : 0u;
      if (!from_local) free_frames(PS, me, ln == 0, tid, wc);  // the root or an exposed task
      const uint32_t have_l = S.ltop - S.lbot;
      uint32_t dry = 0;
      if ((iter & 15u) == 0 && have_l >= 4) {
        if (ln == 0) {
          const int64_t t = static_cast<int64_t>(co_ld64(reinterpret_cast<const uint64_t *>(&cl_deque(p, me)->top)));
          S.top_seen = t;
          dry = (S.bottom - t <= 0) ? 1u : 0u;
        }
        dry = uniform(dry);
      }
      // expose the oldest entries when the stack would overflow or the deque is dry
      uint32_t E = (have_l + k > kBlkLocal) ? (have_l + k - kBlkLocal) : 0u;
      if (dry && have_l / 2 > E) E = have_l / 2;
      if (E > have_l) E = have_l;
      bool ok = true;
      if (E > 0) {
        uint32_t room = 1;
        if (ln == 0) room = cl_room(p, S, me, E) ? 1u : 0u;
        ok = uniform(room) != 0;
        if (!ok) {
          if (ln == 0) raise_error(p, -6 /*GTAP_E_CAPACITY*/, 2, p.cap, E, me, static_cast<int32_t>(job));
        } else {
          const int64_t bot = S.bottom;
          const uint32_t lb = S.lbot;
          for (uint32_t i0 = 0; i0 < E; i0 += kWave) {
            const uint32_t chunk = (E - i0) < kWave ? (E - i0) : kWave;
            AllocResult ar{};
            if (!alloc_frames(p, PS, me, chunk, ar, wc)) {
              ok = false;
              break;
            }
            wave_sync();
            if (ln < chunk) {
              const uint32_t i = i0 + ln;
              const uint32_t e = (lb + i) & (kBlkLocal - 1);
              const uint4 a = S.lstk[2 * e], b = S.lstk[2 * e + 1];
              const uint32_t cid = alloc_id(PS, ar, ln);
              uint64_t *f64 = frame64(frame_ptr(p, cid));
              co_st64(f64 + 0, pack(a.x, a.y));
              co_st64(f64 + 1, pack(a.z, a.w));
              co_st64(f64 + 2, pack(b.x, b.y));
              co_st64(f64 + 3, pack(b.z, b.w));
              co_st32(cl_buf(p, me) + (static_cast<uint64_t>(bot + i) & (p.cap - 1)), cid);
            }
          }
          if (ok) {
            drain();  // frames and slots complete before the deque grows
            if (ln == 0) {
              co_st64(reinterpret_cast<uint64_t *>(&cl_deque(p, me)->bottom), static_cast<uint64_t>(bot + E));
              S.bottom = bot + E;
              S.lbot = lb + E;
            }
            wc.add(ST_PUSHED, E);
          }
        }
        wave_sync();
      }
      if (ok) {
        const uint32_t lt = S.ltop;
        if (ln < k) {
          const uint32_t e = (lt + ln) & (kBlkLocal - 1);
          S.lstk[2 * e] = make_uint4(kNone, job, state_word(TK_FMM, 0, 0), S.child[ln][0]);
          S.lstk[2 * e + 1] = make_uint4(S.child[ln][1], 0, 0, 0);
        }
        wave_sync();
        if (ln == 0) {
          S.ltop = lt + k;
          if (cjob != job) {
            cflush(false);
            cjob = job;
          }
          cdelta += static_cast<int64_t>(k) - 1;
          cflush(true);
        }
        wc.add(ST_SPAWNS, k);
        wc.add(ST_LOCAL, k);
      }
      if (ln == 0) {
        S.next = kNone;
        S.next_cont = 0;
      }
    } else if (wv == 0) {
      const uint32_t out = S.out_type;
      uint32_t next = kNone, next_cont = 0;
      if (out == OUT_FORK) {
        const uint32_t nc = S.nchild;
        if (nc > kMaxChildren) {
          if (ln == 0) raise_error(p, -6 /*GTAP_E_CAPACITY*/, 4, kMaxChildren, nc, me, static_cast<int32_t>(job));
        } else {
          uint32_t *f = frame_ptr(p, tid);
          if (ln == 0) {
            co_st64(reinterpret_cast<uint64_t *>(f + FW_JOIN), static_cast<uint64_t>(nc));
            co_st64(reinterpret_cast<uint64_t *>(f + FW_BIGACC), 0ull);
          }
          // children 1..nc-1 go to the deque, child 0 runs next
          bool ok = true;
          if (ln == 0) ok = cl_room(p, S, me, nc - 1);
          ok = uniform(static_cast<uint32_t>(ok)) != 0;
          if (!ok) {
            if (ln == 0) raise_error(p, -6 /*GTAP_E_CAPACITY*/, 2, p.cap, nc, me, static_cast<int32_t>(job));
          } else {
            const uint32_t ckind = kind;
            const uint32_t state = state_word(ckind, 0, 0);
            const int64_t bot = S.bottom;
            uint32_t first = kNone;
            for (uint32_t done = 0; done < nc && ok; done += kWave) {
              const uint32_t chunk = (nc - done) < kWave ? (nc - done) : kWave;
              AllocResult ar{};
              if (!alloc_frames(p, PS, me, chunk, ar, wc)) {
                ok = false;
                break;
              }
              wave_sync();
              uint32_t cid = kNone;
              if (ln < chunk) {
                const uint32_t g = done + ln;
                cid = alloc_id(PS, ar, ln);
                ChildInit ci{};
                if (ckind == TK_FIB) {
                  ci.p[0] = S.fw[FW_P0] - 1 - g;
                } else if (ckind == TK_UTS) {
                  const uint64_t cidv = split_id(pack(S.fw[FW_P0], S.fw[FW_P0 + 1]), g);
                  ci.p[0] = static_cast<uint32_t>(cidv);
                  ci.p[1] = static_cast<uint32_t>(cidv >> 32);
                  ci.p[2] = S.fw[FW_P0 + 2] + 1;
                  ci.p[3] = S.fw[FW_P0 + 3];
                  ci.p[4] = S.fw[FW_P0 + 4];
                } else {
                  ci.p[0] = S.child[g][0];
                  ci.p[1] = S.child[g][1];
                }
                write_frame(frame_ptr(p, cid), tid, job, state, ci);
                // child 0 runs next on this workgroup, the others go to the deque
                if (g > 0) co_st32(cl_buf(p, me) + (static_cast<uint64_t>(bot + g - 1) & (p.cap - 1)), cid);
              }
              if (done == 0) first = uniform(static_cast<uint32_t>(__shfl(static_cast<int>(cid), 0, 64)));
            }
            if (ok) {
              drain();  // frames and slots complete before the deque grows
              if (ln == 0 && nc > 1) {
                co_st64(reinterpret_cast<uint64_t *>(&cl_deque(p, me)->bottom), static_cast<uint64_t>(bot + nc - 1));
                S.bottom = bot + nc - 1;
              }
              next = first;
              wc.add(ST_SPAWNS, nc);
              wc.add(ST_PUSHED, nc - 1);
            }
          }
        }
      } else {
        // completion; an empty continuation completes the parent in place
        const bool empty_cont = (kind == TK_FMM);
        uint32_t cur = tid;
        uint32_t par = S.fw[FW_PARENT];
        int64_t val = S.value;
        for (;;) {
          free_frames((cur & kBigBit) ? PB : PS, me, ln == 0, cur, wc);
          if (par == kNone) {
            if (ln == 0) {
              store_result(p, job, val);
              drain();
              fetch_add_relaxed(&p.ctl->jobs_remaining, -1);
            }
            break;
          }
          uint32_t resumed = 0, gp = kNone;
          if (ln == 0) {
            uint32_t *pf = frame_ptr(p, par);
            const int64_t lim = static_cast<int64_t>(1) << kSmallValueBits;
            int64_t delta = -1;
            if (val >= lim || val <= -lim) {
              fetch_add_relaxed(bigacc_ptr(pf), val);
              drain();
            } else {
              delta = val * (static_cast<int64_t>(1) << kJoinBits) - 1;
            }
            const int64_t old = fetch_add_relaxed(join_ptr(pf), delta);
            if ((static_cast<uint64_t>(old) & kJoinMask) == 1u) {
              resumed = 1;
              if (empty_cont) gp = co_ld32(pf + FW_PARENT);
            }
          }
          resumed = uniform(resumed);
          if (!resumed) break;
          if (!empty_cont) {
            next = par;
            next_cont = 1;
            break;
          }
          gp = uniform(gp);
          cur = par;
          par = gp;
          val = 0;
          wc.add(ST_CONTS, 1);
        }
      }
      if (ln == 0) {
        S.next = next;
        S.next_cont = next_cont;
      }
    }
    __syncthreads();
    tid = S.next;
    cont = S.next_cont;
    const uint64_t now = clock64();
    busy_cycles += now - t_loop;
    t_loop = now;
  }

  fmm_flush_acc<NT>(S, true, true);
  fmm_flush(p, fc);
  if (tx == 0) {
    for (int i = 0; i < static_cast<int>(ST_COUNT); ++i)
      if (wc.v[i]) fetch_add_relaxed(&p.ctl->stats[i], static_cast<uint64_t>(wc.v[i]));
    if (busy_cycles) fetch_add_relaxed(&p.ctl->stats[ST_BUSY_CYCLES], busy_cycles);
    if (idle_cycles) fetch_add_relaxed(&p.ctl->stats[ST_IDLE_CYCLES], idle_cycles);
  }
}

}  // namespace gtap
