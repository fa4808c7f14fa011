// fmm_lists.h -- the FMM pipeline of GTaP Sec. 6.4.1: the dual-tree traversal
// only builds interaction lists (well-separated cell pairs for M2L, leaf
// pairs for P2P) in fixed-capacity arrays appended with atomic adds; the lists
// are then evaluated by data-parallel kernels.  Two traversals build them:
// thread-mode tasks of the runtime (one cell pair per task, see tasks.h) and a
// level-synchronous worklist (ping-pong frontiers, one launch per frontier).
//
// MI355X choices: appends are aggregated per wavefront (one atomic per
// wavefront and list); the lists are sorted by target cell.  M2L gives each
// target one wavefront, one source per lane, and adds its sums once.  P2P is
// balanced over the list entries instead (64 per wavefront), because a target
// leaf's segment can be tens of thousands of entries long; the wavefronts
// that share a target add their potentials with fp64 atomics.
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

constexpr uint32_t kM2LThreads = 64;

GTAP_DEV double mfact(int t) {  // e_t! = e_x! e_y! e_z! of coefficient t
  const double f[kP + 1] = {1.0, 1.0, 2.0, 6.0, 24.0, 120.0, 720.0};
  return f[kTab.e[t][0]] * f[kTab.e[t][1]] * f[kTab.e[t][2]];
}

// Moments scaled for the list M2L: Q'_b = (-1)^|b| Q_b / b! (in place; the
// list pipeline reads the moments only in M2L).
__global__ void k_scale_moments(double *Q, int64_t ncells) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= ncells * kNc) return;
  const int t = static_cast<int>(i % kNc);
  Q[i] *= ((kTab.deg[t] & 1) ? -1.0 : 1.0) / mfact(t);
}

// Scaled Taylor coefficients T'_g = g! T_g of 1/|d + h| at h = 0 (total degree
// <= 6): the Coulomb three-term recurrence multiplied by g! becomes
// T'_g = -[(2n-1) sum_i g_i d_i T'_{g-e_i} + (n-1) sum_i g_i (g_i - 1) T'_{g-2e_i}] / (n r^2),
// n = |g|.  Fully unrolled, T' stays in registers.
GTAP_DEV void taylor_scaled(double d0, double d1, double d2, double *T) {
  const double inv_r2 = 1.0 / (d0 * d0 + d1 * d1 + d2 * d2);
  T[0] = sqrt(inv_r2);
  const double dd[3] = {d0, d1, d2};
#pragma unroll
  for (int t = 1; t < kNc; ++t) {
    const double n = static_cast<double>(kTab.deg[t]);
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double gi = static_cast<double>(kTab.e[t][i]);
      const uint8_t m1 = kTab.dm1[t][i], m2 = kTab.dm2[t][i];
      if (m1 != 0xFF) s1 += gi * dd[i] * T[m1];
      if (m2 != 0xFF) s2 += gi * (gi - 1.0) * T[m2];
    }
    T[t] = -((2.0 * n - 1.0) * s1 + (n - 1.0) * s2) * inv_r2 / n;
  }
}

// M2L over the sorted list: one wavefront per target cell a, one source per
// lane at a time.  With T' and Q' (above), L_a = (1/a!) sum_b T'_{a+b} Q'_b, so
// a lane keeps the source's 84 coefficients T' and its own 84 sums in
// registers and adds T'_{a+b} Q'_b for every (a, b) with |a| + |b| <= 6 --
// 924 fused multiply-adds, all indices compile-time constants, no LDS.  The
// 64 partial sums are combined by lane shuffles and added to L[a] once.
__global__ __launch_bounds__(kM2LThreads) void k_m2l_list(const int32_t *__restrict__ cell,
                                                          const double *__restrict__ Qs, double *L,
                                                          const uint64_t *__restrict__ pairs,
                                                          const uint64_t *__restrict__ seg_lo,
                                                          const uint64_t *__restrict__ seg_hi) {
  const uint32_t a = blockIdx.x;
  const uint64_t lo = seg_lo[a], hi = seg_hi[a];
  if (lo == hi) return;
  const uint32_t ln = threadIdx.x;
  int32_t A[kCellInts];
  load_cell(cell, a, A);
  const double cx = cell_centre(A[1], A[0]), cy = cell_centre(A[2], A[0]), cz = cell_centre(A[3], A[0]);
  double acc[kNc];
#pragma unroll
  for (int t = 0; t < kNc; ++t) acc[t] = 0.0;
  for (uint64_t s = lo + ln; s < hi; s += kM2LThreads) {
    const uint32_t b = static_cast<uint32_t>(pairs[s]);
    int32_t B[kCellInts];
    load_cell(cell, b, B);
    double T[kNc];
    taylor_scaled(cx - cell_centre(B[1], B[0]), cy - cell_centre(B[2], B[0]), cz - cell_centre(B[3], B[0]), T);
    const double *q = Qs + static_cast<size_t>(b) * kNc;
#pragma unroll
    for (int tb = 0; tb < kNc; ++tb) {
      const double qb = q[tb];
#pragma unroll
      for (int ta = 0; ta < ncoef(kP - kTab.deg[tb]); ++ta)
        acc[ta] += T[kTab.idx[kTab.e[ta][0] + kTab.e[tb][0]][kTab.e[ta][1] + kTab.e[tb][1]]
                             [kTab.e[ta][2] + kTab.e[tb][2]]] * qb;
    }
  }
#pragma unroll
  for (int t = 0; t < kNc; ++t) {
    double v = acc[t];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if (ln == 0) L[static_cast<size_t>(a) * kNc + t] += v / mfact(t);
  }
}

constexpr uint32_t kP2PThreads = 256;
constexpr uint32_t kP2PTileL = 64;

// 1 / sqrt(x) for x > 0: the hardware estimate refined by two Newton-Raphson
// steps y <- y (3 - x y^2) / 2 (each squares the relative error).
GTAP_DEV double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}

// P2P over the sorted list, balanced over its entries: wavefront w takes the
// 64 entries 64 w .. 64 w + 63 (one per lane), so a target whose segment is
// long (a large leaf next to a dense region meets tens of thousands of source
// leaves) is spread over many wavefronts, and adds its potentials atomically.
// The entries form runs of one target.  Per run, the sources of its leaves
// are concatenated (exclusive prefix of the leaf sizes over the run's lanes)
// and walked in chunks of 64 points: the owner of chunk position c is the
// last leaf starting at or before it (marks in LDS and a prefix maximum), each
// lane loads one point, the chunk is staged in LDS as (x, y, z, q), and the
// next chunk is loaded while this one is evaluated.  A tile of at most 64
// targets is padded to a power of two P; the lanes form 64 / P groups of P
// (lane = target + P * group), group g takes the chunk's sources g, g + 64/P,
// ..., and the groups' partial sums meet by lane shuffles.  Interactions are
// counted, and coincident pairs as the pairs at distance zero less the
// points' meetings with themselves (one per target point and self pair).
__global__ __launch_bounds__(kP2PThreads) void k_p2p_list(const int32_t *__restrict__ cell,
                                                          const double *__restrict__ px,
                                                          const double *__restrict__ py,
                                                          const double *__restrict__ pz,
                                                          const double *__restrict__ pq, double *phi,
                                                          const uint64_t *__restrict__ pairs, uint64_t n,
                                                          uint32_t ncells, uint64_t *inter_out, uint64_t *coinc_out) {
  constexpr uint32_t W = kP2PThreads / kWave;
  __shared__ double2 stage[W][2 * kWave];
  __shared__ uint32_t mark[W][kWave];
  const uint32_t tx = threadIdx.x, ln = tx % kWave;
  const uint32_t wv = __builtin_amdgcn_readfirstlane(tx / kWave);
  const uint64_t e0 = (static_cast<uint64_t>(blockIdx.x) * W + wv) * kWave;
  if (e0 >= n) return;
  const uint32_t ne = static_cast<uint32_t>(min(static_cast<uint64_t>(kWave), n - e0));
  double2 *const st = stage[wv];
  uint32_t *const mk = mark[wv];
  // entry e0 + ln: target ta (ncells for the gaps, which sort last, and past
  // the end), source leaf sb with points rb .. rb + rn - 1, target points
  // tb .. tb + tn - 1
  uint32_t ta = ncells, sb = 0;
  int32_t rb = 0, rn = 0, tb = 0, tn = 0;
  if (ln < ne) {
    const uint64_t e = pairs[e0 + ln];
    if (static_cast<uint32_t>(e >> 32) < ncells) {
      ta = static_cast<uint32_t>(e >> 32);
      sb = static_cast<uint32_t>(e);
      rb = cell[static_cast<size_t>(sb) * kCellInts + 4];
      rn = cell[static_cast<size_t>(sb) * kCellInts + 5] - rb;
      tb = cell[static_cast<size_t>(ta) * kCellInts + 4];
      tn = cell[static_cast<size_t>(ta) * kCellInts + 5] - tb;
    }
  }
  const uint32_t nv = static_cast<uint32_t>(__popcll(ballot(ta < ncells)));
  uint64_t inter = 0, selfm = 0;
  uint32_t zc = 0;
  for (uint32_t k0 = 0; k0 < nv;) {
    // the run of target a: lanes k0 .. k1 - 1
    const uint32_t a = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(ta), static_cast<int>(k0)));
    const uint64_t other = ballot(ta != a) & (~0ull << k0);
    const uint32_t k1 = other ? static_cast<uint32_t>(__builtin_ctzll(other)) : kWave;
    const bool in_run = ln >= k0 && ln < k1;
    const int32_t rn_run = in_run ? rn : 0;
    const int32_t incl = static_cast<int32_t>(wave_inclusive_sum(static_cast<uint32_t>(rn_run)));
    const int32_t pre = incl - rn_run;  // first concatenated position of this lane's leaf
    const int32_t stotal = __builtin_amdgcn_readlane(incl, static_cast<int>(k1 - 1));
    const int32_t ab = __builtin_amdgcn_readlane(tb, static_cast<int>(k0));
    const int32_t na = __builtin_amdgcn_readlane(tn, static_cast<int>(k0));
    const uint32_t nself = static_cast<uint32_t>(__popcll(ballot(in_run && sb == a)));
    inter += static_cast<uint64_t>(static_cast<int64_t>(na) * stotal - static_cast<int64_t>(nself) * na);
    selfm += static_cast<uint64_t>(nself) * static_cast<uint64_t>(na);
    // Loads chunk c's points into (sx, sy, sz, sq).
    double sx = 0.0, sy = 0.0, sz = 0.0, sq = 0.0;
    auto fetch = [&](int32_t c) {
      mk[ln] = 0;
      wave_sync();
      if (in_run && rn > 0 && pre < c + static_cast<int32_t>(kWave) && pre + rn > c)
        mk[pre > c ? pre - c : 0] = ln + 1;
      wave_sync();
      const uint32_t m = wave_inclusive_max(mk[ln]);
      wave_sync();
      const int32_t own = m ? static_cast<int32_t>(m) - 1 : 0;
      const int32_t ob = __shfl(rb, own, 64), op = __shfl(pre, own, 64);
      const int32_t pos = c + static_cast<int32_t>(ln);
      if (pos < stotal) {
        const int32_t sj = ob + (pos - op);
        sx = px[sj];
        sy = py[sj];
        sz = pz[sj];
        sq = pq[sj];
      }
    };
    for (int32_t t0 = 0; t0 < na; t0 += static_cast<int32_t>(kP2PTileL)) {
      const int32_t nt = min(static_cast<int32_t>(kP2PTileL), na - t0);
      uint32_t P = 1;
      while (P < static_cast<uint32_t>(nt)) P <<= 1;
      const int32_t ng = static_cast<int32_t>(kWave / P);
      const uint32_t tl = ln % P;
      const int32_t grp = static_cast<int32_t>(ln / P);
      const int32_t i = ab + t0 + static_cast<int32_t>(tl);
      const bool live = static_cast<int32_t>(tl) < nt;
      double xi = live ? px[i] : 0.0, yi = live ? py[i] : 0.0, zi = live ? pz[i] : 0.0;
      // taken as written here, so that the source loop's waits do not cover
      // the source prefetch
      asm volatile("" : "+v"(xi), "+v"(yi), "+v"(zi));
      double acc = 0.0;
      fetch(0);
      for (int32_t c0 = 0; c0 < stotal; c0 += static_cast<int32_t>(kWave)) {
        const int32_t cnt = min(static_cast<int32_t>(kWave), stotal - c0);
        if (static_cast<int32_t>(ln) < cnt) {
          st[2 * ln] = make_double2(sx, sy);
          st[2 * ln + 1] = make_double2(sz, sq);
        }
        wave_sync();
        if (c0 + static_cast<int32_t>(kWave) < stotal) fetch(c0 + static_cast<int32_t>(kWave));
#pragma unroll 4
        for (int32_t u = 0; u < cnt; u += ng) {
          // u + grp < 64: u is a multiple of ng below cnt <= 64, grp < ng
          const int32_t j = u + grp;
          const bool ok = j < cnt;
          const double2 s01 = st[2 * j], s23 = st[2 * j + 1];
          const double dx = xi - s01.x, dy = yi - s01.y, dz = zi - s23.x;
          const double r2 = dx * dx + dy * dy + dz * dz;
          const bool z = r2 == 0.0;
          const double ri = rsqrt_nr(z ? 1.0 : r2);
          acc += (ok && !z) ? s23.y * ri : 0.0;
          zc += (ok && z && live) ? 1u : 0u;
        }
        wave_sync();  // the chunk's reads are issued before the next one overwrites it
      }
      for (uint32_t d = P; d < kWave; d <<= 1) acc += __shfl_xor(acc, static_cast<int>(d), 64);
      if (live && grp == 0) unsafeAtomicAdd(phi + i, acc);
    }
    k0 = k1;
  }
  const uint64_t coinc = readlane64(wave_inclusive_sum64(zc), 63) - selfm;
  if (ln == 0 && inter) fetch_add_relaxed(inter_out, inter);
  if (ln == 0 && coinc) fetch_add_relaxed(coinc_out, coinc);
}

}  // namespace fmm
}  // namespace gtap
