// tasks.h -- thread-mode task bodies as hand-written resumable state machines.
//
// The paper's compiler turns a pragma-annotated task function into one that
// stores join-crossing values in its task record and, when re-invoked,
// switches on the saved resume point (Sec. 5.2).  Here every task kind is
// written in that lowered form by hand: exec_task() reads the frame, switches
// on (kind, resume point) and reports one of
//   OUT_DONE  -- the task returned `value` (to its parent, or as the job result)
//   OUT_FORK  -- the task spawned `nchild` children described by `d[]` and
//                suspended at its join; the runtime sets the waiting-child
//                counter and re-executes the frame at resume point 1 after the
//                last child completed (Sec. 5.1.2).
// Children are materialised later, by the whole wavefront, from the
// descriptor: make_child() builds child j of a forked parent.  A child's
// arguments are copied into its own frame at spawn time (firstprivate
// semantics, Sec. 4.1).  Each task has an implicit join at its end, so a
// parent always completes after all of its children.
#pragma once
#include "fmm_lists.h"
#include "kclique_bits.h"
#include "layout.h"
#include "wave.h"

namespace gtap {

enum OutType : uint32_t { OUT_NONE = 0, OUT_DONE = 1, OUT_FORK = 2 };

// N 32-bit words kept in aligned 64-bit slots.  Every access is a whole-slot
// read or read-modify-write, so no two accesses to the array partly overlap
// (the optimizer merges two adjacent 32-bit stores of one 64-bit value into a
// single 64-bit store; at an odd word offset that overlaps two slots and keeps
// the array in memory -- here it would go to LDS -- instead of registers).
template <uint32_t N>
struct Words {
  uint64_t w[(N + 1) / 2];
  struct Ref {
    uint64_t &s;
    uint32_t hi;
    GTAP_DEV operator uint32_t() const { return static_cast<uint32_t>(hi ? (s >> 32) : s); }
    GTAP_DEV Ref &operator=(uint32_t v) {
      s = hi ? ((s & 0xFFFFFFFFull) | (static_cast<uint64_t>(v) << 32)) : ((s & ~0xFFFFFFFFull) | v);
      return *this;
    }
    GTAP_DEV Ref &operator=(const Ref &r) { return *this = static_cast<uint32_t>(r); }
  };
  GTAP_DEV Ref operator[](uint32_t i) { return Ref{w[i >> 1], i & 1u}; }
  GTAP_DEV uint32_t operator[](uint32_t i) const {
    return static_cast<uint32_t>((i & 1u) ? (w[i >> 1] >> 32) : w[i >> 1]);
  }
};

struct Outcome {
  uint32_t type;
  uint32_t nchild;   // OUT_FORK: number of children
  uint32_t big;      // OUT_FORK: children need big frames
  uint32_t ckind;    // OUT_FORK: children's task kind
  Words<6> d;        // OUT_FORK: child-generation descriptor
  int64_t value;     // OUT_DONE: return value
  uint32_t parent;   // parent task ID (kNone for a root)
  uint32_t job;
  uint32_t kind;     // this task's kind
  uint32_t first;    // 1: first execution (resume point 0), 0: continuation
  uint32_t emit;     // FMM list traversal: 1 = M2L pair, 2 = P2P pair (d[0], d[1]), descriptor d[3..4]
  uint32_t pc_next;  // OUT_FORK of the extended kinds: resume point after the join (Cilksort sorts fork twice)
  uint32_t words;    // 4-byte words of task data the body read or wrote (k-clique lists), for the byte count
};

// Payload of a new frame (words 3..7).
struct ChildInit {
  Words<kPayloadWords> p;
};

GTAP_DEV uint32_t *frame_ptr(const Params &p, uint32_t tid) {
  return (tid & kBigBit) ? p.frames_b + static_cast<size_t>(tid & ~kBigBit) * p.stride_b
                         : p.frames_s + static_cast<size_t>(tid) * kFrameWords;
}
GTAP_DEV uint64_t *frame64(uint32_t *f) { return reinterpret_cast<uint64_t *>(f); }
GTAP_DEV int64_t *join_ptr(uint32_t *f) { return reinterpret_cast<int64_t *>(f + FW_JOIN); }
GTAP_DEV int64_t *bigacc_ptr(uint32_t *f) { return reinterpret_cast<int64_t *>(f + FW_BIGACC); }

GTAP_DEV uint32_t state_word(uint32_t kind, uint32_t pc, uint32_t cls) {
  return kind | (pc << 8) | (cls << 16);
}
GTAP_DEV uint64_t pack(uint32_t lo, uint32_t hi) {
  return static_cast<uint64_t>(lo) | (static_cast<uint64_t>(hi) << 32);
}

// Spawn-time frame image: four coherent 64-bit stores.
GTAP_DEV void write_frame(uint32_t *f, uint32_t parent, uint32_t job, uint32_t state,
                          const ChildInit &c) {
  uint64_t *f64 = frame64(f);
  co_st64(f64 + 0, pack(parent, job));
  co_st64(f64 + 1, pack(state, c.p[0]));
  co_st64(f64 + 2, pack(c.p[1], c.p[2]));
  co_st64(f64 + 3, pack(c.p[3], c.p[4]));
}

// splitmix64 output function (Steele, Lea, Flood, OOPSLA 2014), from its
// published definition: add the golden gamma, two xor-shift-multiply rounds,
// a final xor-shift.
GTAP_DEV uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// Child i of a node: mix64 of the parent id advanced by (i+1) gammas.
GTAP_DEV uint64_t split_id(uint64_t a, uint64_t i) { return mix64(a + (i + 1) * 0x9E3779B97F4A7C15ull); }

// Geometric child count: leading draws j = 1, 2, ... whose hash is below thr.
// Four draws per round: they are independent, so their multiply chains
// overlap; the count is the index of the first failed draw all the same.
GTAP_DEV uint32_t uts_children(uint64_t id, uint32_t depth, uint64_t thr, uint32_t max_depth) {
  if (depth >= max_depth) return 0;
  constexpr uint64_t kStep = 0xD1B54A32D192ED03ull;
  for (uint32_t c = 0;; c += 4) {
    const uint64_t j = c + 1;
    const bool a0 = mix64(id ^ (j * kStep)) < thr;
    const bool a1 = mix64(id ^ ((j + 1) * kStep)) < thr;
    const bool a2 = mix64(id ^ ((j + 2) * kStep)) < thr;
    const bool a3 = mix64(id ^ ((j + 3) * kStep)) < thr;
    if (!a0) return c;
    if (!a1) return c + 1;
    if (!a2) return c + 2;
    if (!a3) return c + 3;
  }
}

// First index in the ascending list b[lo, nb) whose element is >= x, by a
// galloping search (doubling steps from lo, then bisection), and in *v that
// element (when the index is below nb: every candidate for the answer was
// loaded on the way, so the caller needs no second load of it); kCo: b is
// read coherently (a buffer another wavefront wrote).
template <bool kCo>
GTAP_DEV int32_t ld_list(const int32_t *b, uint32_t i) {
  if constexpr (kCo) return co_ld32i(b + i);
  else return b[i];
}
template <bool kCo>
GTAP_DEV uint32_t gallop_list(const int32_t *b, uint32_t lo, uint32_t nb, int32_t x, int32_t *v) {
  if (lo >= nb) return nb;
  const int32_t y = ld_list<kCo>(b, lo);
  if (y >= x) {
    *v = y;
    return lo;
  }
  uint32_t step = 1, prev = lo;
  int32_t vh = 0;
  while (prev + step < nb) {
    const int32_t t = ld_list<kCo>(b, prev + step);
    if (t >= x) {
      vh = t;
      break;
    }
    prev += step;
    step <<= 1;
  }
  uint32_t l = prev + 1, h = prev + step < nb ? prev + step : nb;
  while (l < h) {
    const uint32_t mid = l + (h - l) / 2;
    const int32_t t = ld_list<kCo>(b, mid);
    if (t < x) {
      l = mid + 1;
    } else {
      h = mid;
      vh = t;
    }
  }
  *v = vh;
  return l;
}
// Common elements of the ascending lists s (walked) and l (galloped into);
// the next element of s is loaded while the current one's search runs.
template <bool kCoS, bool kCoL>
GTAP_DEV uint32_t isect_gallop(const int32_t *s, uint32_t ns, const int32_t *l, uint32_t nl, int32_t *out) {
  uint32_t j = 0, o = 0;
  int32_t x = ld_list<kCoS>(s, 0);
  for (uint32_t i = 0; i < ns && j < nl; ++i) {
    const int32_t xn = i + 1 < ns ? ld_list<kCoS>(s, i + 1) : 0;
    int32_t v = 0;
    j = gallop_list<kCoL>(l, j, nl, x, &v);
    if (j < nl && v == x) {
      if (out) co_st32i(out + o, x);
      ++o;
      ++j;
    }
    x = xn;
  }
  return o;
}

// |C /\ B| for an ascending candidate list C (read coherently: it may be a
// buffer another wavefront wrote) and an ascending CSR list B (read-only
// input); writes the intersection coherently if out != 0.  The shorter list
// is walked and each of its elements galloped to in the longer one.
GTAP_DEV uint32_t intersect_sorted(const int32_t *C, uint32_t nc, const int32_t *B, uint32_t nb,
                                   int32_t *out) {
  if (nc == 0 || nb == 0) return 0;
  return nc <= nb ? isect_gallop<true, false>(C, nc, B, nb, out) : isect_gallop<false, true>(B, nb, C, nc, out);
}

// Job arguments.  Read coherently: while serving, a job slot is rewritten by
// the wave that admits the next job using it.
GTAP_DEV uint64_t job_arg(const Params &p, uint32_t job, uint32_t i) { return co_ld64(&p.jobs[job].a[i]); }

// Words 0..7 of a task: its frame's first half, or the LDS descriptor of a
// task that has no frame (a child retained by the wavefront that spawned it).
struct TaskImage {
  uint64_t w01, w23, w45, w67;
};

GTAP_DEV TaskImage load_image(const Params &p, uint32_t tid) {
  const uint64_t *f64 = frame64(frame_ptr(p, tid));
  return TaskImage{co_ld64(f64 + 0), co_ld64(f64 + 1), co_ld64(f64 + 2), co_ld64(f64 + 3)};
}

// A resumed parent needs its header and its join state only; all four loads
// go out together.  w45/w67 carry the join word and the large-value sum.
GTAP_DEV TaskImage load_continuation(const Params &p, uint32_t tid) {
  uint32_t *f = frame_ptr(p, tid);
  const uint64_t *f64 = frame64(f);
  return TaskImage{co_ld64(f64 + 0), co_ld64(f64 + 1), static_cast<uint64_t>(ld_relaxed(join_ptr(f))),
                   static_cast<uint64_t>(ld_relaxed(bigacc_ptr(f)))};
}

// ---------------------------------------------------------------------------
// Cilksort pieces (Sec. 6.3).  Buffers: job argument 0 = keys, 1 = scratch;
// a task's destination bit picks one, its sources are in the other.  Keys
// pass between tasks that may run on different XCDs, so they are read and
// written with device-coherent accesses (and the scheduler drains a
// wavefront's writes before its completions reach the join words).
constexpr uint32_t kSortNet = 64;            // serial sorts: a 64-wide network
constexpr uint32_t kMergeD = (1u << 29) - 1;  // merge payload word 4: destination start

// Bitonic sorting network on 64 keys held in registers (all indices are
// compile-time constants after unrolling, so nothing spills to scratch).
GTAP_DEV void sort_net64(uint32_t *v) {
#pragma unroll
  for (uint32_t k = 2; k <= kSortNet; k <<= 1) {
#pragma unroll
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (uint32_t i = 0; i < kSortNet; ++i) {
        const uint32_t l = i ^ j;
        if (l > i) {
          const uint32_t lo = v[i] < v[l] ? v[i] : v[l], hi = v[i] < v[l] ? v[l] : v[i];
          const bool up = (i & k) == 0;
          v[i] = up ? lo : hi;
          v[l] = up ? hi : lo;
        }
      }
    }
  }
}

// Number of keys of the sorted range s[0, n) below v.
GTAP_DEV uint32_t count_below(const uint32_t *s, uint32_t n, uint32_t v) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = lo + (hi - lo) / 2;
    if (co_ld32(s + mid) < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// k-clique counting with bitset candidate subgraphs and cost-threshold
// splitting (Sec. 6.4.2); the encoding is described in kclique_bits.h.  Job
// arguments: 0 row_ptr, 1 col, 2 n, 3 k, 4 range_leaf, 5 max out-degree,
// 6 threshold | algorithm << 8 (0 orientation, 1 pivoting).
struct KsJob {
  const int32_t *rp;
  const int32_t *col;
  uint64_t *mat;   // job argument 7: n+1 vertex offsets, then the bit matrices
  uint32_t n;
  uint32_t kk;     // k - 2: clique size inside an edge's candidate set
  uint32_t thr;
  bool pivot;
};
GTAP_DEV KsJob ks_job(const Params &p, uint32_t job) {
  const uint64_t a6 = job_arg(p, job, 6);
  return KsJob{reinterpret_cast<const int32_t *>(job_arg(p, job, 0)),
               reinterpret_cast<const int32_t *>(job_arg(p, job, 1)),
               reinterpret_cast<uint64_t *>(job_arg(p, job, 7)), static_cast<uint32_t>(job_arg(p, job, 2)),
               static_cast<uint32_t>(job_arg(p, job, 3)) - 2, static_cast<uint32_t>(a6 & 0xFFu),
               ((a6 >> 8) & 1u) != 0};
}

// Vertex u's bit matrices: D (row i: the members of N+(u) that are
// out-neighbours of its i-th member), then for pivoting U (D or its
// transpose); d x W words each.  The offsets are read coherently like all
// job data.
struct KsMat {
  uint64_t *D;
  uint64_t *rows;  // the rows the search uses: U for pivoting, else D
  uint32_t d, W;
};
GTAP_DEV KsMat ks_mat(const KsJob &J, uint32_t u) {
  const uint32_t d = static_cast<uint32_t>(J.rp[u + 1] - J.rp[u]);
  const uint32_t W = (d + 63) / 64;
  uint64_t *D = J.mat + (J.n + 1) + co_ld64(J.mat + u);
  return KsMat{D, J.pivot ? D + static_cast<size_t>(d) * W : D, d, W};
}

// Store a node's state at buf (device-coherent: its children read it).
GTAP_DEV void ks_store_node(uint32_t *buf, uint64_t meta, const uint64_t *P, const uint64_t *R, uint32_t W,
                            bool with_r) {
  uint64_t *b = reinterpret_cast<uint64_t *>(buf);
  co_st64(b, meta);
  for (uint32_t w = 0; w < W; ++w) co_st64(b + 1 + w, P[w]);
  if (with_r)
    for (uint32_t w = 0; w < W; ++w) co_st64(b + 1 + W + w, R[w]);
}

// Pivot of a split pivoting node: the member of P with the most neighbours in
// P, the lowest on ties; R receives its non-neighbours other than itself.
GTAP_DEV uint32_t ks_pivot(const uint64_t *rows, uint32_t W, const uint64_t *P, uint64_t *R) {
  uint32_t best = 0;
  int32_t bd = -1;
  for (uint32_t w = 0; w < W; ++w) {
    for (uint64_t t = P[w]; t; t &= t - 1) {
      const uint32_t x = w * 64 + __builtin_ctzll(t);
      int32_t d = 0;
      for (uint32_t v = 0; v < W; ++v) d += __popcll(P[v] & co_ld64(rows + static_cast<size_t>(x) * W + v));
      if (d > bd) {
        bd = d;
        best = x;
      }
    }
  }
  for (uint32_t v = 0; v < W; ++v) R[v] = P[v] & ~co_ld64(rows + static_cast<size_t>(best) * W + v);
  R[best >> 6] &= ~(1ull << (best & 63));
  return best;
}

// Row task (u, i): row i of u's matrix, from N+(u) /\ N+(x), x = N+(u)[i],
// galloping from the shorter list; for pivoting also ORed into U both ways
// (U was cleared by the vertex task).
GTAP_DEV void ks_row(const Params &p, Outcome &o, uint32_t u, uint32_t i) {
  const KsJob J = ks_job(p, o.job);
  const KsMat M = ks_mat(J, u);
  const uint32_t d = M.d, W = M.W;
  const int32_t *nu = J.col + J.rp[u];
  const int32_t x = nu[i];
  const int32_t *nx = J.col + J.rp[x];
  const uint32_t dx = static_cast<uint32_t>(J.rp[x + 1] - J.rp[x]);
  uint64_t *D = M.D + static_cast<size_t>(i) * W;
  uint64_t *U = M.rows;
  o.words = 4 + d + dx + (J.pivot ? 4 : 2) * W;  // row bounds, both lists, the row (and U's) written
  uint32_t cw = 0;
  uint64_t acc = 0;
  auto flush = [&]() {  // word cw of row i is complete
    co_st64(D + cw, acc);
    if (J.pivot && acc) fetch_or_relaxed(U + static_cast<size_t>(i) * W + cw, acc);
    ++cw;
    acc = 0;
  };
  auto hit = [&](uint32_t j) {  // j ascending
    while ((j >> 6) > cw) flush();
    acc |= 1ull << (j & 63);
    if (J.pivot) fetch_or_relaxed(U + static_cast<size_t>(j) * W + (i >> 6), static_cast<uint64_t>(1) << (i & 63));
  };
  if (d <= dx) {  // each member of N+(u), galloped to in N+(x)
    uint32_t t = 0;
    for (uint32_t j = 0; j < d && t < dx; ++j) {
      t = kcs::gallop(nx, t, dx, nu[j]);
      if (t < dx && nx[t] == nu[j]) {
        hit(j);
        ++t;
      }
    }
  } else {  // each out-neighbour of x, galloped to in N+(u)
    uint32_t j = 0;
    for (uint32_t t = 0; t < dx && j < d; ++t) {
      j = kcs::gallop(nu, j, d, nx[t]);
      if (j < d && nu[j] == nx[t]) {
        hit(j);
        ++j;
      }
    }
  }
  while (cw < W) flush();
}

// A vertex with d <= threshold out-neighbours (k >= 4): its matrix in private
// one-word rows (galloping as the row tasks do), then every edge's search in
// place: edge i's candidates are row i.
GTAP_DEV int64_t ks_vertex_in_place(const KsJob &J, uint32_t u, uint32_t d, uint32_t &words) {
  const int32_t *nu = J.col + J.rp[u];
  uint64_t A[kcs::kMaxThr], B[kcs::kMaxThr];
  words += d;
  for (uint32_t i = 0; i < d; ++i) {
    const int32_t x = nu[i];
    const int32_t *nx = J.col + J.rp[x];
    const uint32_t dx = static_cast<uint32_t>(J.rp[x + 1] - J.rp[x]);
    words += 2 + dx;
    uint64_t r = 0;
    if (d <= dx) {
      uint32_t t = 0;
      for (uint32_t j = 0; j < d && t < dx; ++j) {
        t = kcs::gallop(nx, t, dx, nu[j]);
        if (t < dx && nx[t] == nu[j]) {
          r |= 1ull << j;
          ++t;
        }
      }
    } else {
      uint32_t j = 0;
      for (uint32_t t = 0; t < dx && j < d; ++t) {
        j = kcs::gallop(nu, j, d, nx[t]);
        if (j < d && nu[j] == nx[t]) {
          r |= 1ull << j;
          ++j;
        }
      }
    }
    A[i] = r;
    B[i] = r;
  }
  if (J.pivot)  // both directions
    for (uint32_t i = 0; i < d; ++i)
      for (uint64_t t = A[i]; t; t &= t - 1) B[__builtin_ctzll(t)] |= 1ull << i;
  int64_t total = 0;
  for (uint32_t i = 0; i < d; ++i) {
    if (static_cast<uint32_t>(__popcll(A[i])) < J.kk) continue;
    total += J.pivot ? kcs::sct_count(B, A[i], 0, 0, J.kk) : kcs::dag_count(A, A[i], J.kk);
  }
  return total;
}

// Edge task (u, i): the i-th out-neighbour v of u.  k = 3: |N+(u) /\ N+(v)|.
// Otherwise its candidates are row i of u's matrix: few -> renumbered into a
// private one-word matrix and counted in place; more than the threshold ->
// one child task takes the search over.
GTAP_DEV void ks_edge(const Params &p, Outcome &o, uint32_t u, uint32_t i) {
  const KsJob J = ks_job(p, o.job);
  if (J.kk == 1) {
    const int32_t s0 = J.rp[u];
    const int32_t v = J.col[s0 + i];
    const uint32_t du = static_cast<uint32_t>(J.rp[u + 1] - s0), dv = static_cast<uint32_t>(J.rp[v + 1] - J.rp[v]);
    o.words = 5 + du + dv;
    o.value = kcs::isect(J.col + s0, du, J.col + J.rp[v], dv, nullptr, 0);
    return;
  }
  const KsMat M = ks_mat(J, u);
  const uint32_t W = M.W;
  o.words = 4 + 2 * W;  // row bounds, matrix offset, the edge's row
  uint64_t S[kcs::kMaxW];
  uint32_t c = 0;
  for (uint32_t w = 0; w < W; ++w) {
    S[w] = co_ld64(M.D + static_cast<size_t>(i) * W + w);
    c += __popcll(S[w]);
  }
  if (c < J.kk) return;
  if (!J.pivot && J.kk == 2) {  // directed edges inside C
    o.words += 2 * W * c;  // the candidates' rows
    int64_t e = 0;
    for (uint32_t w = 0; w < W; ++w)
      for (uint64_t t = S[w]; t; t &= t - 1) {
        const uint32_t y = w * 64 + __builtin_ctzll(t);
        for (uint32_t v = 0; v < W; ++v) e += __popcll(S[v] & co_ld64(M.D + static_cast<size_t>(y) * W + v));
      }
    o.value = e;
    return;
  }
  if (c > J.thr) {
    o.type = OUT_FORK;
    o.nchild = 1;
    o.ckind = TK_KS_HEAVY;
    o.big = 1;
    o.d[0] = u;
    o.d[1] = i;
    return;
  }
  uint64_t A[kcs::kMaxThr];
  o.words += 2 * W * c;  // the candidates' rows
  kcs::compact(M.rows, W, S, A);
  const uint64_t all = kcs::low_mask(c);
  o.value = J.pivot ? kcs::sct_count(A, all, 0, 0, J.kk) : kcs::dag_count(A, all, J.kk);
}

// Root node of a heavy edge's search (its big frame holds the node state;
// the matrix is u's): one task per branch.
GTAP_DEV void ks_heavy(const Params &p, uint32_t *f, Outcome &o, uint32_t u, uint32_t i) {
  const KsJob J = ks_job(p, o.job);
  const KsMat M = ks_mat(J, u);
  const uint32_t W = M.W;
  uint64_t P[kcs::kMaxW], R[kcs::kMaxW];
  uint32_t c = 0;
  for (uint32_t w = 0; w < W; ++w) {
    P[w] = co_ld64(M.D + static_cast<size_t>(i) * W + w);
    c += __popcll(P[w]);
  }
  uint64_t meta = J.kk;
  uint32_t nchild = c;
  o.words = 4 + 2 * W + (J.pivot ? 2 * W * (c + 1) + 2 + 4 * W : 2 + 2 * W);  // row; pivot rows; node state
  if (J.pivot) {
    const uint32_t piv = ks_pivot(M.rows, W, P, R);
    meta = static_cast<uint64_t>(piv) << 32;  // no held vertices, no pivots yet
    nchild = 1;
    for (uint32_t w = 0; w < W; ++w) nchild += __popcll(R[w]);
  }
  ks_store_node(f + FW_BUF, meta, P, R, W, J.pivot);
  o.type = OUT_FORK;
  o.nchild = nchild;
  o.ckind = TK_KS_NODE;
  o.big = (J.pivot || J.kk - 1 >= 3) ? 1u : 0u;  // children that may split keep state in a big frame
  o.d[0] = u;
  o.d[1] = 0;
}

// Branch j of a node that split: u is the vertex whose matrix the search
// uses, ns the node state's offset in the parent's buffer.
GTAP_DEV void ks_node(const Params &p, uint32_t *f, Outcome &o, uint32_t u, uint32_t j, uint32_t ns) {
  const KsJob J = ks_job(p, o.job);
  const KsMat M = ks_mat(J, u);
  const uint32_t W = M.W;
  const uint64_t *rows = M.rows;
  const uint64_t *pb = reinterpret_cast<const uint64_t *>(frame_ptr(p, o.parent) + FW_BUF + ns);
  const uint64_t meta = co_ld64(pb);
  uint64_t P[kcs::kMaxW], S[kcs::kMaxW], R[kcs::kMaxW];
  for (uint32_t w = 0; w < W; ++w) P[w] = co_ld64(pb + 1 + w);
  o.words = 6 + 4 * W;  // row bounds, matrix offset, node meta and set, one row
  uint32_t m = 0;
  uint64_t A[kcs::kMaxThr];
  if (!J.pivot) {
    const uint32_t l = static_cast<uint32_t>(meta & 0xFFFFu) - 1;
    const uint32_t x = kcs::select_bit(P, W, j);
    for (uint32_t w = 0; w < W; ++w) {
      S[w] = P[w] & co_ld64(rows + static_cast<size_t>(x) * W + w);
      m += __popcll(S[w]);
    }
    if (l == 1) {
      o.value = m;
      return;
    }
    if (m < l) return;
    o.words += 2 * W * m;  // the rows of the node's candidates
    if (l == 2) {  // directed edges inside S
      int64_t e = 0;
      for (uint32_t w = 0; w < W; ++w)
        for (uint64_t t = S[w]; t; t &= t - 1) {
          const uint32_t y = w * 64 + __builtin_ctzll(t);
          for (uint32_t v = 0; v < W; ++v) e += __popcll(S[v] & co_ld64(rows + static_cast<size_t>(y) * W + v));
        }
      o.value = e;
      return;
    }
    if (m <= J.thr) {
      kcs::compact(rows, W, S, A);
      o.value = kcs::dag_count(A, kcs::low_mask(m), l);
      return;
    }
    ks_store_node(f + FW_BUF, l, S, S, W, false);
    o.type = OUT_FORK;
    o.nchild = m;
    o.big = l - 1 >= 3 ? 1u : 0u;  // level <= 2 is always counted in place
  } else {
    uint32_t h = static_cast<uint32_t>(meta & 0xFFFFu), q = static_cast<uint32_t>((meta >> 16) & 0xFFFFu);
    const uint32_t piv = static_cast<uint32_t>(meta >> 32);
    if (j == 0) {  // the pivot branch
      for (uint32_t w = 0; w < W; ++w) S[w] = P[w] & co_ld64(rows + static_cast<size_t>(piv) * W + w);
      q += 1;
    } else {  // the (j-1)-th non-neighbour of the pivot, held
      for (uint32_t w = 0; w < W; ++w) R[w] = co_ld64(pb + 1 + W + w);
      const uint32_t x = kcs::select_bit(R, W, j - 1);
      for (uint32_t w = 0; w < W; ++w) {
        const uint64_t before = w < (x >> 6) ? R[w] : w == (x >> 6) ? (R[w] & kcs::low_mask(x & 63)) : 0ull;
        S[w] = P[w] & ~before & co_ld64(rows + static_cast<size_t>(x) * W + w);
      }
      S[piv >> 6] &= ~(1ull << (piv & 63));
      h += 1;
    }
    for (uint32_t w = 0; w < W; ++w) m += __popcll(S[w]);
    if (h == J.kk) {
      o.value = 1;
      return;
    }
    if (m == 0) {
      o.value = kcs::binom(q, J.kk - h);
      return;
    }
    if (m + q < J.kk - h) return;
    o.words += 2 * W * (m + (j == 0 ? 0 : 1));  // the candidates' rows (and R)
    if (m <= J.thr) {
      kcs::compact(rows, W, S, A);
      o.value = kcs::sct_count(A, kcs::low_mask(m), h, q, J.kk);
      return;
    }
    const uint32_t np = ks_pivot(rows, W, S, R);
    ks_store_node(f + FW_BUF, h | (static_cast<uint64_t>(q) << 16) | (static_cast<uint64_t>(np) << 32), S, R, W,
                  true);
    uint32_t nchild = 1;
    for (uint32_t w = 0; w < W; ++w) nchild += __popcll(R[w]);
    o.type = OUT_FORK;
    o.nchild = nchild;
    o.big = 1;
  }
  o.ckind = TK_KS_NODE;
  o.d[0] = u;
  o.d[1] = 0;
}

// ---------------------------------------------------------------------------
// Execute one task on this lane.  tid is its frame, or kNone for a task
// without one (then it runs at resume point 0 and needs no buffer).  kExt
// adds the extension task sets it names (instantiated separately, so the
// other task kinds compile unchanged).
template <uint32_t kExt = 0>
GTAP_DEV void exec_task(const Params &p, uint32_t tid, const TaskImage &img, Outcome &o) {
  uint32_t *f = tid != kNone ? frame_ptr(p, tid) : nullptr;
  const uint64_t w01 = img.w01;
  const uint64_t w23 = img.w23;
  const uint32_t state = static_cast<uint32_t>(w23);
  const uint32_t kind = state & 0xFFu;
  const uint32_t pc = (state >> 8) & 0xFFu;
  o.parent = static_cast<uint32_t>(w01);
  o.job = static_cast<uint32_t>(w01 >> 32);
  o.kind = kind;
  o.first = pc == 0 ? 1u : 0u;
  o.type = OUT_DONE;
  o.nchild = 0;
  o.big = 0;
  o.value = 0;
  if constexpr (kExt) {
    o.emit = 0;
    o.pc_next = 1;
    if constexpr ((kExt & kExtLists) != 0) {
      if (pc != 0 && kind == TK_SORT) {
        // after the two sorts: merge them back (resume point 2 follows); after
        // the merge: done, the result is the range's length
        uint32_t *f = frame_ptr(p, tid);
        const uint32_t lo = co_ld32(f + FW_P0), n = co_ld32(f + FW_P0 + 1), dst = co_ld32(f + FW_P0 + 2);
        if (pc == 1) {
          const uint32_t h = n / 2;
          o.type = OUT_FORK;
          o.nchild = 1;
          o.ckind = TK_MERGE;
          o.d[0] = lo; o.d[1] = h; o.d[2] = lo + h; o.d[3] = n - h; o.d[4] = lo | (dst << 31); o.d[5] = 0;
          o.pc_next = 2;
          return;
        }
        o.value = n;
        return;
      }
    }
    if constexpr ((kExt & kExtSplit) != 0) {
      if (pc == 1 && kind == TK_KS_VERTEX) {  // the matrix is complete: the edge tasks
        const uint32_t u = co_ld32(frame_ptr(p, tid) + FW_P0);  // (written at spawn or when it forked)
        const int32_t *rp = reinterpret_cast<const int32_t *>(job_arg(p, o.job, 0));
        o.type = OUT_FORK;
        o.nchild = static_cast<uint32_t>(rp[u + 1] - rp[u]);
        o.ckind = TK_KS_EDGE;
        o.d[0] = u;
        o.pc_next = 2;
        return;
      }
    }
  }

  if (pc != 0) {
    // Continuation after the join (image from load_continuation): every kind
    // sums its children's results; a UTS node adds itself.
    const int64_t acc = (static_cast<int64_t>(img.w45) >> kJoinBits) + static_cast<int64_t>(img.w67);
    o.value = (kind == TK_UTS) ? acc + 1 : acc;
    return;
  }

  const uint64_t w45 = img.w45;
  const uint64_t w67 = img.w67;
  const uint32_t p0 = static_cast<uint32_t>(w23 >> 32);
  const uint32_t p1 = static_cast<uint32_t>(w45), p2 = static_cast<uint32_t>(w45 >> 32);
  const uint32_t p3 = static_cast<uint32_t>(w67), p4 = static_cast<uint32_t>(w67 >> 32);
  if constexpr (kExt) {
    if constexpr ((kExt & kExtLists) != 0) {
      if (kind == TK_SORT) {
        // sort(lo, n, dst): serial below the cutoff, else both halves into the
        // other buffer first (resume point 1 merges them)
        const uint32_t lo = p0, n = p1, dst = p2;
        const uint32_t sc = static_cast<uint32_t>(job_arg(p, o.job, 3));
        if (n <= sc) {
          const uint32_t *X = reinterpret_cast<const uint32_t *>(job_arg(p, o.job, 0));
          uint32_t *D = reinterpret_cast<uint32_t *>(job_arg(p, o.job, dst ? 1 : 0));
          uint32_t v[kSortNet];
  #pragma unroll
          for (uint32_t i = 0; i < kSortNet; ++i) v[i] = i < n ? co_ld32(X + lo + i) : 0xFFFFFFFFu;
          sort_net64(v);
  #pragma unroll
          for (uint32_t i = 0; i < kSortNet; ++i)
            if (i < n) co_st32(D + lo + i, v[i]);
          o.value = n;
          return;
        }
        o.type = OUT_FORK;
        o.nchild = 2;
        o.ckind = TK_SORT;
        o.d[0] = lo; o.d[1] = n; o.d[2] = dst;
        return;
      }
      if (kind == TK_MERGE) {
        // merge(A, B -> D): payload A = (p0, p1), B = (p2, p3), p4 = destination
        // start | split pending << 29 | side << 30 | destination buffer << 31.
        // A pending split first takes its side of the parent's ranges.
        uint32_t a0 = p0, na = p1, b0 = p2, nb = p3;
        const uint32_t dst = p4 >> 31;
        uint32_t d0 = p4 & kMergeD;
        const uint32_t *S = reinterpret_cast<const uint32_t *>(job_arg(p, o.job, dst ? 0 : 1));
        uint32_t *D = reinterpret_cast<uint32_t *>(job_arg(p, o.job, dst ? 1 : 0));
        if ((p4 >> 29) & 1u) {
          const uint32_t ma = na / 2, mb = count_below(S + b0, nb, co_ld32(S + a0 + ma));
          if ((p4 >> 30) & 1u) {
            a0 += ma; na -= ma; b0 += mb; nb -= mb; d0 += ma + mb;
          } else {
            na = ma; nb = mb;
          }
        }
        if (nb > na) {
          const uint32_t t0 = a0, t1 = na;
          a0 = b0; na = nb; b0 = t0; nb = t1;
        }
        const uint32_t mc = static_cast<uint32_t>(job_arg(p, o.job, 3) >> 32);
        if (na + nb <= mc) {
          uint32_t i = 0, j = 0, k = d0;
          while (i < na && j < nb) {
            const uint32_t x = co_ld32(S + a0 + i), y = co_ld32(S + b0 + j);
            if (y < x) {
              co_st32(D + k++, y);
              ++j;
            } else {
              co_st32(D + k++, x);
              ++i;
            }
          }
          while (i < na) co_st32(D + k++, co_ld32(S + a0 + i++));
          while (j < nb) co_st32(D + k++, co_ld32(S + b0 + j++));
          return;
        }
        o.type = OUT_FORK;
        o.nchild = 2;
        o.ckind = TK_MERGE;
        o.d[0] = a0; o.d[1] = na; o.d[2] = b0; o.d[3] = nb; o.d[4] = d0 | (dst << 31); o.d[5] = 1;
        return;
      }
    }
    if constexpr ((kExt & kExtSplit) != 0) {
      if (kind == TK_KS_RANGE) {  // vertex range: halves, then one vertex task per vertex
        const uint32_t lo = p0, hi = p1;
        const uint32_t leaf = static_cast<uint32_t>(job_arg(p, o.job, 4));
        if (hi <= lo) return;
        o.type = OUT_FORK;
        o.d[0] = lo; o.d[1] = hi;
        o.nchild = hi - lo > leaf ? 2 : hi - lo;
        o.ckind = hi - lo > leaf ? TK_KS_RANGE : TK_KS_VERTEX;
        return;
      }
      if (kind == TK_KS_VERTEX) {
        // k = 3: one edge task per out-neighbour.  k >= 4 (at least k-1
        // out-neighbours): the row tasks of the vertex's matrix first (resume
        // point 1 forks the edge tasks, resume point 2 sums them)
        const int32_t *rp = reinterpret_cast<const int32_t *>(job_arg(p, o.job, 0));
        const uint32_t k = static_cast<uint32_t>(job_arg(p, o.job, 3));
        const uint32_t deg = static_cast<uint32_t>(rp[p0 + 1] - rp[p0]);
        o.words = 2;
        if (k <= 2) {
          o.value = k == 1 ? 1 : deg;
          return;
        }
        if (deg == 0 || (k >= 4 && deg < k - 1)) return;
        o.type = OUT_FORK;
        o.nchild = deg;
        o.d[0] = p0;
        if (k == 3) {  // no matrix: the edge tasks now, the sum at resume point 2
          o.ckind = TK_KS_EDGE;
          o.pc_next = 2;
          return;
        }
        const KsJob J = ks_job(p, o.job);
        if (deg <= J.thr) {  // few out-neighbours: the whole vertex in place, one-word rows
          o.type = OUT_DONE;
          o.value = ks_vertex_in_place(J, p0, deg, o.words);
          return;
        }
        if (J.pivot) {  // U is built by atomic ORs: cleared first
          const KsMat M = ks_mat(J, p0);
          for (uint32_t x = 0; x < deg * M.W; ++x) co_st64(M.rows + x, 0ull);
          o.words += 2 * deg * M.W;
        }
        o.ckind = TK_KS_ROW;
        return;
      }
      if (kind == TK_KS_ROW) {
        ks_row(p, o, p0, p1);
        return;
      }
      if (kind == TK_KS_EDGE) {
        ks_edge(p, o, p0, p1);
        return;
      }
      if (kind == TK_KS_HEAVY) {
        ks_heavy(p, f, o, p0, p1);
        return;
      }
      if (kind == TK_KS_NODE) {
        ks_node(p, f, o, p0, p1, p2);
        return;
      }
    }
    if constexpr ((kExt & kExtLists) != 0) {
      if (kind == TK_DTT) {
        // FMM cell pair (A, B) (Sec. 6.4.1): an accepted pair or a pair of
        // leaves goes to its list (the scheduler appends it, one atomic per
        // wavefront), any other pair forks the pairs of the wider cell's
        // children.  Payload: A, B, descriptor (p2, p3), theta = p4 & 255 over
        // p4 >> 8.
        const fmm::FmmDesc *D = reinterpret_cast<const fmm::FmmDesc *>(pack(p2, p3));
        int32_t A[fmm::kCellInts], B[fmm::kCellInts];
        fmm::load_cell(D->cell, p0, A);
        fmm::load_cell(D->cell, p1, B);
        bool split_a = false;
        const uint32_t dec = fmm::dtt_decide(A, B, static_cast<int64_t>(p4 & 0xFFu), static_cast<int64_t>(p4 >> 8), split_a);
        o.d[0] = p0; o.d[1] = p1; o.d[3] = p2; o.d[4] = p3; o.d[5] = p4;
        if (dec != 0) {
          o.emit = dec;
          return;
        }
        o.type = OUT_FORK;
        o.nchild = static_cast<uint32_t>(split_a ? A[7] : B[7]);
        o.ckind = TK_DTT;
        o.d[2] = static_cast<uint32_t>(split_a ? A[6] : B[6]) | (split_a ? 0x80000000u : 0u);
        return;
      }
    }
  }
  switch (kind) {
    case TK_FIB: {
      // fib(n): n < 2 returns n, else spawn fib(n-1), fib(n-2) and join.
      const uint32_t n = p0;
      if (n < 2) {
        o.value = n;
        return;
      }
      o.type = OUT_FORK;
      o.nchild = 2;
      o.ckind = TK_FIB;
      o.d[0] = n;
      return;
    }
    case TK_NQ: {
      // Rows [0,row) hold queens; one child per unattacked column of `row`.
      // The board size travels in the payload (p4).
      const uint32_t n = p4;
      const uint32_t full = (1u << n) - 1u;
      const uint32_t cols = p0, dl = p1, dr = p2, row = p3;
      if (row == n) {
        o.value = 1;
        return;
      }
      const uint32_t avail = full & ~(cols | dl | dr);
      if (avail == 0) return;  // dead end: 0
      o.type = OUT_FORK;
      o.nchild = __popc(avail);
      o.ckind = TK_NQ;
      o.d[0] = cols; o.d[1] = dl; o.d[2] = dr; o.d[3] = row; o.d[4] = avail; o.d[5] = n;
      return;
    }
    case TK_UTS: {
      // payload: id (p0,p1), depth | depth limit << 16 (p2), threshold (p3,p4)
      const uint64_t id = pack(p0, p1);
      const uint32_t depth = p2 & 0xFFFFu, max_depth = p2 >> 16;
      const uint32_t nc = uts_children(id, depth, pack(p3, p4), max_depth);
      if (nc == 0) {
        o.value = 1;
        return;
      }
      o.type = OUT_FORK;
      o.nchild = nc;
      o.ckind = TK_UTS;
      o.d[0] = p0; o.d[1] = p1; o.d[2] = p2; o.d[3] = p3; o.d[4] = p4;
      return;
    }
    case TK_KC_RANGE: {
      // Vertex range [lo,hi): halve while larger than range_leaf, else one
      // vertex task per vertex.
      const uint32_t lo = p0, hi = p1;
      const uint32_t leaf = static_cast<uint32_t>(job_arg(p, o.job, 4));
      if (hi <= lo) return;
      o.type = OUT_FORK;
      o.d[0] = lo; o.d[1] = hi;
      if (hi - lo > leaf) {
        o.nchild = 2;
        o.ckind = TK_KC_RANGE;
      } else {
        o.nchild = hi - lo;
        o.ckind = TK_KC_VERTEX;
      }
      return;
    }
    case TK_KC_VERTEX: {
      // K(N+(v), k-1): k = 1 counts the vertex, k = 2 its out-degree, else one
      // candidate task per out-neighbour with C = N+(v).
      const int32_t *rp = reinterpret_cast<const int32_t *>(job_arg(p, o.job, 0));
      const int32_t *col = reinterpret_cast<const int32_t *>(job_arg(p, o.job, 1));
      const uint32_t k = static_cast<uint32_t>(job_arg(p, o.job, 3));
      const uint32_t v = p0;
      if (k == 1) {
        o.value = 1;
        return;
      }
      const int32_t s = rp[v], e = rp[v + 1];
      const uint32_t deg = static_cast<uint32_t>(e - s);
      o.words = 2;
      if (k == 2) {
        o.value = deg;
        return;
      }
      if (deg == 0) return;
      const uint64_t cptr = reinterpret_cast<uint64_t>(col + s);
      o.type = OUT_FORK;
      o.nchild = deg;
      o.ckind = TK_KC_CAND;
      o.big = (k - 2 >= 2) ? 1u : 0u;
      o.d[0] = static_cast<uint32_t>(cptr); o.d[1] = static_cast<uint32_t>(cptr >> 32);
      o.d[2] = deg; o.d[3] = k - 2;
      return;
    }
    case TK_KC_CAND: {
      // K(C /\ N+(u), l): l = 1 counts the intersection, else stores it in this
      // frame's buffer and forks one child per element.
      const int32_t *rp = reinterpret_cast<const int32_t *>(job_arg(p, o.job, 0));
      const int32_t *col = reinterpret_cast<const int32_t *>(job_arg(p, o.job, 1));
      const uint32_t u = p0, l = p1;
      const int32_t *C = reinterpret_cast<const int32_t *>(pack(p2, p3));
      const uint32_t nC = p4;
      const int32_t s = rp[u], e = rp[u + 1];
      const uint32_t nu = static_cast<uint32_t>(e - s);
      o.words = 2 + nC + nu;  // row bounds, the parent's candidates, N+(u)
      if (l == 1) {
        o.value = intersect_sorted(C, nC, col + s, nu, nullptr);
        return;
      }
      int32_t *buf = reinterpret_cast<int32_t *>(f + FW_BUF);
      const uint32_t m = intersect_sorted(C, nC, col + s, nu, buf);
      o.words += m;  // the candidates written for the children
      if (m == 0) return;
      const uint64_t cptr = reinterpret_cast<uint64_t>(buf);
      o.type = OUT_FORK;
      o.nchild = m;
      o.ckind = TK_KC_CAND;
      o.big = (l - 1 >= 2) ? 1u : 0u;
      o.d[0] = static_cast<uint32_t>(cptr); o.d[1] = static_cast<uint32_t>(cptr >> 32);
      o.d[2] = m; o.d[3] = l - 1;
      return;
    }
    default:
      return;
  }
}

// ---------------------------------------------------------------------------
// Divergence-Aware Queueing (Sec. 4.2, "The queue Clause"): the class of a new
// child selects the deque it waits in, and every wavefront batch is filled
// from one class.  Continuations (resumed parents) are not queued: they are
// always retained with the batch being formed.
GTAP_DEV uint32_t bucket_of(const Params &p, uint32_t x) {
  uint32_t c = 0;
  while (c + 1 < p.Q && x > static_cast<uint32_t>(p.daq_bounds[c])) ++c;
  return c;
}

// Class of child payload c of kind ckind.  GTAP_DAQ_KCLIQUE: a candidate task
// is classed by min(|C_parent|, outdeg(u)), the spawn-time bound on the size
// of its intersection and thus on its cost; a vertex task by its out-degree
// (its candidate set is N+(v)); a vertex-range task, whose subtree spans many
// vertices, by the highest class.
template <uint32_t kExt = 0>
GTAP_DEV uint32_t child_class(const Params &p, uint32_t job, uint32_t ckind, const ChildInit &c) {
  if (p.Q <= 1) return 0;
  if constexpr (kExt) {
    if constexpr ((kExt & kExtLists) != 0) {
      if (p.daq_policy == 3) {  // Cilksort: recursive 0, serial sort 1, serial merge 2
        const uint64_t cut = job_arg(p, job, 3);
        if (ckind == TK_SORT) return (c.p[1] <= static_cast<uint32_t>(cut) ? 1u : 0u) % p.Q;
        if (ckind == TK_MERGE) {
          const uint32_t m = c.p[1] + c.p[3];  // a pending split takes about half
          const uint32_t est = ((c.p[4] >> 29) & 1u) ? m / 2 : m;
          return (est <= static_cast<uint32_t>(cut >> 32) ? 2u : 0u) % p.Q;
        }
        return 0;
      }
    }
    if constexpr ((kExt & kExtSplit) != 0) {
      if (p.daq_policy == 2 && ckind >= TK_KS_RANGE) {
        // split k-clique: a vertex by its out-degree; an edge by its candidate
        // count when its row of the vertex's matrix is built (k >= 4; its
        // parent forks the edges only then), else by min(outdeg u, outdeg v);
        // ranges, row tasks, a heavy edge's search and its branches in the
        // highest class
        if (ckind != TK_KS_EDGE && ckind != TK_KS_VERTEX) return p.Q - 1;
        const KsJob J = ks_job(p, job);
        const uint32_t u = c.p[0];
        if (ckind == TK_KS_VERTEX) return bucket_of(p, static_cast<uint32_t>(J.rp[u + 1] - J.rp[u]));
        if (J.kk >= 2) {
          const KsMat M = ks_mat(J, u);
          uint32_t n = 0;
          for (uint32_t w = 0; w < M.W; ++w) n += __popcll(co_ld64(M.D + static_cast<size_t>(c.p[1]) * M.W + w));
          return bucket_of(p, n);
        }
        const int32_t v = J.col[J.rp[u] + c.p[1]];
        const uint32_t du = static_cast<uint32_t>(J.rp[u + 1] - J.rp[u]), dv = static_cast<uint32_t>(J.rp[v + 1] - J.rp[v]);
        return bucket_of(p, du < dv ? du : dv);
      }
    }
  }
  switch (p.daq_policy) {
    case 1: {  // by kind
      const uint32_t k = ckind == TK_FIB ? 0u : ckind == TK_NQ ? 1u : ckind == TK_UTS ? 2u : 3u;
      return k % p.Q;
    }
    case 2: {  // k-clique candidate-set bound
      if (ckind == TK_KC_RANGE) return p.Q - 1;
      const int32_t *rp = reinterpret_cast<const int32_t *>(job_arg(p, job, 0));
      if (ckind == TK_KC_VERTEX) {
        const uint32_t v = c.p[0];
        return bucket_of(p, static_cast<uint32_t>(rp[v + 1] - rp[v]));
      }
      if (ckind != TK_KC_CAND) return 0;
      const uint32_t u = c.p[0], nC = c.p[4];
      const uint32_t deg = static_cast<uint32_t>(rp[u + 1] - rp[u]);
      return bucket_of(p, deg < nC ? deg : nC);
    }
    default:
      return 0;
  }
}

GTAP_DEV uint32_t nth_set_bit(uint32_t m, uint32_t j) {
  for (uint32_t i = 0; i < j; ++i) m &= m - 1;
  return m & (0u - m);
}

// Payload of child j of a forked parent with child kind `ckind` and
// descriptor d.
template <uint32_t kExt = 0>
GTAP_DEV void make_child(uint32_t ckind, const Words<6> &d, uint32_t j, ChildInit &c) {
  for (uint32_t i = 0; i < kPayloadWords; ++i) c.p[i] = 0;
  if constexpr (kExt) {
    if constexpr ((kExt & kExtLists) != 0) {
      if (ckind == TK_SORT) {  // half j into the other buffer
        const uint32_t h = d[1] / 2;
        c.p[0] = d[0] + (j ? h : 0u);
        c.p[1] = j ? d[1] - h : h;
        c.p[2] = d[2] ^ 1u;
        return;
      }
      if (ckind == TK_MERGE) {  // d[5] = 0: the merge of a sort; 1: side j of a split
        c.p[0] = d[0]; c.p[1] = d[1]; c.p[2] = d[2]; c.p[3] = d[3];
        c.p[4] = d[5] ? (d[4] | (1u << 29) | (j << 30)) : d[4];
        return;
      }
    }
    if constexpr ((kExt & kExtSplit) != 0) {
      if (ckind == TK_KS_RANGE) {
        const uint32_t lo = d[0], hi = d[1], mid = lo + (hi - lo) / 2;
        c.p[0] = j == 0 ? lo : mid;
        c.p[1] = j == 0 ? mid : hi;
        return;
      }
      if (ckind == TK_KS_VERTEX) {
        c.p[0] = d[0] + j;
        return;
      }
      if (ckind == TK_KS_EDGE || ckind == TK_KS_ROW) {  // (u, index of the out-neighbour)
        c.p[0] = d[0];
        c.p[1] = j;
        return;
      }
      if (ckind == TK_KS_HEAVY) {  // the only child: the forking edge's own (u, index)
        c.p[0] = d[0];
        c.p[1] = d[1];
        return;
      }
      if (ckind == TK_KS_NODE) {  // (vertex, branch, parent's node-state offset)
        c.p[0] = d[0];
        c.p[1] = j;
        c.p[2] = d[1];
        return;
      }
    }
    if constexpr ((kExt & kExtLists) != 0) {
      if (ckind == TK_DTT) {  // pair (child j of the split cell, the other cell)
        const bool sa = (d[2] >> 31) != 0;
        const uint32_t c0 = d[2] & 0x7FFFFFFFu;
        c.p[0] = sa ? c0 + j : d[0];
        c.p[1] = sa ? d[1] : c0 + j;
        c.p[2] = d[3];
        c.p[3] = d[4];
        c.p[4] = d[5];
        return;
      }
    }
  }
  switch (ckind) {
    case TK_FIB:
      c.p[0] = d[0] - 1 - j;
      break;
    case TK_NQ: {
      const uint32_t b = nth_set_bit(d[4], j);
      const uint32_t full = (1u << d[5]) - 1u;
      c.p[0] = d[0] | b;
      c.p[1] = ((d[1] | b) << 1) & full;
      c.p[2] = (d[2] | b) >> 1;
      c.p[3] = d[3] + 1;
      c.p[4] = d[5];
      break;
    }
    case TK_UTS: {
      const uint64_t cid = split_id(pack(d[0], d[1]), j);
      c.p[0] = static_cast<uint32_t>(cid);
      c.p[1] = static_cast<uint32_t>(cid >> 32);
      c.p[2] = d[2] + 1;  // depth + 1, depth limit unchanged in the high half
      c.p[3] = d[3];
      c.p[4] = d[4];
      break;
    }
    case TK_KC_RANGE: {
      const uint32_t lo = d[0], hi = d[1], mid = lo + (hi - lo) / 2;
      c.p[0] = j == 0 ? lo : mid;
      c.p[1] = j == 0 ? mid : hi;
      break;
    }
    case TK_KC_VERTEX:
      c.p[0] = d[0] + j;
      break;
    case TK_KC_CAND: {
      const int32_t *C = reinterpret_cast<const int32_t *>(pack(d[0], d[1]));
      c.p[0] = static_cast<uint32_t>(co_ld32i(C + j));
      c.p[1] = d[3];
      c.p[2] = d[0];
      c.p[3] = d[1];
      c.p[4] = d[2];
      break;
    }
    default:
      break;
  }
}

}  // namespace gtap
