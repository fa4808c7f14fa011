// fmm_eval.h -- evaluation of the sorted FMM interaction lists (GTaP Sec.
// 6.4.1 names the phases): M2L into the local expansions, P2P into the
// potentials.  The lists come from the traversals of fmm_lists.h, sorted by
// target cell.
//
// MI355X choices: M2L gives each target one wavefront, one source per lane,
// and adds its sums once.  P2P is balanced over the list entries instead (64
// per wavefront), because a target leaf's segment can be tens of thousands of
// entries long; the wavefronts that share a target add their potentials with
// fp64 atomics.
#pragma once
#include "fmm_lists.h"

namespace gtap {
namespace fmm {

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
