// kclique_bits.h -- k-clique counting with bitset-encoded candidate subgraphs
// and cost-threshold task splitting (Sec. 6.4.2, orientation and pivoting).
//
// Every k-clique is counted at the edge (u, v) between its two lowest vertices
// in the orientation's order; its other k-2 vertices form a (k-2)-clique of
// the edge's candidate set C = N+(u) /\ N+(v).  A vertex task u encodes the
// subgraph induced on N+(u) (d vertices, ascending) as a bit matrix: row i
// holds the members of N+(u) that are out-neighbours of its i-th member, in
// W = ceil(d/64) words; its row tasks build the rows in parallel.  Edge (u, v)
// then finds C as v's row, and the adjacency inside C in the rows of C's
// members -- out-neighbours for the orientation algorithm, neighbours in
// either direction (a second matrix, U) for pivoting.
//
// A node of the search splits when its candidate set is larger than the
// threshold t (the spawn-time cost estimate): it stores its state in its frame
// and forks one task per branch, and every child applies the same test.  A
// node at or below the threshold is finished by one lane in place: its
// candidates are renumbered into a private 64 x 64 matrix (one word per row)
// and the recursion runs on registers and a private stack.
//
//   orientation   node (S, l) counts l-cliques of the DAG on S:
//                 K(S,1) = |S|, K(S,l) = sum over x in S of K(S /\ row x, l-1)
//   pivoting      node (P, h, q) of the succinct clique tree (Jain and
//                 Seshadhri, WSDM 2020): h held vertices, q pivots, candidates
//                 P.  Leaves add binom(q, k-2-h); the pivot p is the candidate
//                 with the most neighbours in P (lowest index on ties); the
//                 branches are p as a pivot, then each non-neighbour w of p in
//                 ascending order as a held vertex, with the candidates that
//                 remain after removing p and the earlier non-neighbours.
//
// The bit matrices of all vertices of a job live in one device buffer the
// library allocates per run, after n+1 per-vertex offsets (64-bit words)
// computed on the host from row_ptr: vertex u's D, then for pivoting its U.
// A node task's big-frame buffer holds only its node state: one 64-bit meta
// word (level or held count | pivots << 16 | pivot << 32), the candidate set
// P (W words), pivoting's branch set R (W words: the pivot's non-neighbours
// other than the pivot).
// Data another task reads (matrices, node state) is stored with
// device-coherent stores (U by device-scope atomic ORs onto a cleared matrix)
// and read with device-coherent loads.
#pragma once
#include "layout.h"
#include "wave.h"

namespace gtap {
namespace kcs {

constexpr uint32_t kMaxW = 16;            // words per row: out-degrees <= 1024
constexpr uint32_t kMaxThr = 64;          // in-place node sets fit one word
constexpr uint32_t kMaxK = 32;            // clique size
constexpr uint32_t kStack = kMaxThr + 2;  // in-place pivoting depth bound

// Big-frame buffer ints of a node task (its node state) for out-degree
// bound D.
__host__ __device__ inline uint32_t buffer_ints(uint32_t D) {
  const uint32_t W = D > 0 ? (D + 63) / 64 : 1;
  return 2 + 4 * W;
}

GTAP_DEV uint64_t low_mask(uint32_t m) { return m >= 64 ? ~0ull : ((1ull << m) - 1); }

// Position of the j-th set bit (from 0) of a W-word set.
GTAP_DEV uint32_t select_bit(const uint64_t *s, uint32_t W, uint32_t j) {
  for (uint32_t w = 0; w < W; ++w) {
    uint64_t t = s[w];
    const uint32_t n = __popcll(t);
    if (j < n) {
      for (uint32_t i = 0; i < j; ++i) t &= t - 1;
      return w * 64 + __builtin_ctzll(t);
    }
    j -= n;
  }
  return 0;
}

// binom(n, r), exact whenever the result fits in 64 bits: C(n-r+i, i) from
// C(n-r+i-1, i-1) times (n-r+i) over i; a large partial value is divided by
// its common factor with i first, after which i's remaining factor divides
// (n-r+i).
GTAP_DEV uint64_t gcd64(uint64_t a, uint64_t b) {
  while (b) {
    const uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}
GTAP_DEV int64_t binom(uint32_t n, uint32_t r) {
  if (r > n) return 0;
  if (r > n - r) r = n - r;
  uint64_t v = 1;
  for (uint32_t i = 1; i <= r; ++i) {
    const uint64_t b = n - r + i;
    if (v < (1ull << 52)) {
      v = v * b / i;
    } else {
      const uint64_t g = gcd64(v, i);
      v = (v / g) * (b / (i / g));
    }
  }
  return static_cast<int64_t>(v);
}

// First index in the ascending b[lo, nb) whose element is >= x: a galloping
// search from lo (doubling steps, then bisection), cheap when the answer is
// near lo.
GTAP_DEV uint32_t gallop(const int32_t *b, uint32_t lo, uint32_t nb, int32_t x) {
  if (lo >= nb || b[lo] >= x) return lo;
  uint32_t step = 1, prev = lo;  // b[prev] < x
  while (prev + step < nb && b[prev + step] < x) {
    prev += step;
    step <<= 1;
  }
  uint32_t l = prev + 1, h = prev + step < nb ? prev + step : nb;  // answer in [l, h]
  while (l < h) {
    const uint32_t mid = l + (h - l) / 2;
    if (b[mid] < x) l = mid + 1;
    else h = mid;
  }
  return l;
}

// Size of the intersection of two ascending lists (read-only graph data);
// the first `cap` common elements go to out (ascending).  Each element of the
// shorter list is galloped to in the longer one: a lane's search is a chain of
// dependent loads, and on the skewed degrees of power-law graphs galloping
// needs far fewer of them than a merge.
GTAP_DEV uint32_t isect(const int32_t *a, uint32_t na, const int32_t *b, uint32_t nb, int32_t *out, uint32_t cap) {
  const int32_t *s = na < nb ? a : b, *l = na < nb ? b : a;
  const uint32_t ns = na < nb ? na : nb, nl = na < nb ? nb : na;
  uint32_t j = 0, o = 0;
  for (uint32_t i = 0; i < ns && j < nl; ++i) {
    const int32_t x = s[i];
    j = gallop(l, j, nl, x);
    if (j < nl && l[j] == x) {
      if (o < cap) out[o] = x;
      ++o;
      ++j;
    }
  }
  return o;
}

// l-cliques of the DAG with one-word rows A on the set S0 (orientation, in place).
GTAP_DEV int64_t dag_count(const uint64_t *A, uint64_t S0, uint32_t l) {
  if (l == 1) return __popcll(S0);
  int64_t total = 0;
  if (l == 2) {
    for (uint64_t t = S0; t; t &= t - 1) total += __popcll(S0 & A[__builtin_ctzll(t)]);
    return total;
  }
  uint64_t sS[kMaxK], sRem[kMaxK];
  uint32_t sp = 0, d = l;  // counting d-cliques of S; rem: members not expanded yet
  uint64_t S = S0, rem = S0;
  for (;;) {
    if (rem == 0) {
      if (sp == 0) return total;
      --sp;
      S = sS[sp];
      rem = sRem[sp];
      ++d;
      continue;
    }
    const uint32_t x = __builtin_ctzll(rem);
    rem &= rem - 1;
    const uint64_t T = S & A[x];
    if (d == 3) {  // pairs inside T, directly
      for (uint64_t t = T; t; t &= t - 1) total += __popcll(T & A[__builtin_ctzll(t)]);
      continue;
    }
    if (static_cast<uint32_t>(__popcll(T)) < d - 1) continue;
    sS[sp] = S;
    sRem[sp] = rem;
    ++sp;
    S = T;
    rem = T;
    --d;
  }
}

// k'-cliques below the clique-tree node (P0, h0, q0) with one-word undirected
// rows A (pivoting, in place).
GTAP_DEV int64_t sct_count(const uint64_t *A, uint64_t P0, uint32_t h0, uint32_t q0, uint32_t kk) {
  uint64_t sP[kStack], sR[kStack];
  uint32_t sHQ[kStack];
  int64_t total = 0;
  uint32_t sp = 0;
  uint64_t P = P0;
  uint32_t h = h0, q = q0;
  for (;;) {
    // enter node (P, h, q)
    if (h == kk) {
      total += 1;
    } else if (P == 0) {
      total += binom(q, kk - h);
    } else if (static_cast<uint32_t>(__popcll(P)) + q >= kk - h) {
      uint32_t best = 0;
      int32_t bd = -1;
      for (uint64_t t = P; t; t &= t - 1) {
        const uint32_t x = __builtin_ctzll(t);
        const int32_t dx = __popcll(P & A[x]);
        if (dx > bd) {
          bd = dx;
          best = x;
        }
      }
      const uint64_t pb = 1ull << best;
      sP[sp] = P & ~pb;
      sR[sp] = P & ~A[best] & ~pb;
      sHQ[sp] = h | (q << 16);
      ++sp;
      P &= A[best];  // first branch: the pivot
      q += 1;
      continue;
    }
    // leave: next branch of the innermost open node
    for (;;) {
      if (sp == 0) return total;
      const uint64_t Rr = sR[sp - 1];
      if (Rr == 0) {
        --sp;
        continue;
      }
      const uint32_t w = __builtin_ctzll(Rr);
      sR[sp - 1] = Rr & (Rr - 1);
      const uint64_t Pc = sP[sp - 1];
      sP[sp - 1] = Pc & ~(1ull << w);
      P = Pc & A[w];
      h = (sHQ[sp - 1] & 0xFFFFu) + 1;
      q = sHQ[sp - 1] >> 16;
      break;
    }
  }
}

// Renumber the members of the W-word set s (at most 64 of them) into one-word
// rows A, from the c x W matrix `rows` (device-coherent reads).  Returns the
// member count.
GTAP_DEV uint32_t compact(const uint64_t *rows, uint32_t W, const uint64_t *s, uint64_t *A) {
  uint32_t pre[kMaxW];
  uint32_t m = 0;
  for (uint32_t w = 0; w < W; ++w) {
    pre[w] = m;
    m += __popcll(s[w]);
  }
  uint32_t a = 0;
  for (uint32_t w = 0; w < W; ++w) {
    for (uint64_t t = s[w]; t; t &= t - 1) {
      const uint32_t x = w * 64 + __builtin_ctzll(t);
      uint64_t r = 0;
      for (uint32_t v = 0; v < W; ++v) {
        uint64_t u = co_ld64(rows + static_cast<size_t>(x) * W + v) & s[v];
        for (; u; u &= u - 1) {
          const uint32_t b = __builtin_ctzll(u);
          r |= 1ull << (pre[v] + __popcll(s[v] & low_mask(b)));
        }
      }
      A[a++] = r;
    }
  }
  return m;
}

}  // namespace kcs
}  // namespace gtap
