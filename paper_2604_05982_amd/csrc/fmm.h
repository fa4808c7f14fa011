// fmm.h -- 3D Laplace FMM for block mode: octree construction, upward and
// downward passes as data-parallel kernels, and the cell-pair work that the
// dual-tree traversal tasks run (GTaP Sec. 6.4.1).
//
// Conventions (the paper names the phases only):
//   * root cube [-2^7, 2^7)^3; grid coordinate floor((x + 2^7) * 2^13) in
//     [0, 2^21); 63-bit Morton key (bit 3k+2: x, 3k+1: y, 3k: z); points sorted
//     by (key, index);
//   * a cell splits iff it holds more than leaf_max points below level 21;
//     only non-empty children; cells numbered level by level in Morton order;
//   * MAC theta = ta/tb on doubled integer centres:
//     accept iff 3 tb^2 (w_A + w_B)^2 < ta^2 |C2_A - C2_B|^2;
//   * Cartesian Taylor expansions of 1/|x - y| of total degree <= 6:
//     moments Q_b = sum q (y - c_B)^b, locals
//     L_a = sum_b C(a+b, a) (-1)^|b| T_{a+b}(c_A - c_B) Q_b, where T_g are the
//     Taylor coefficients of 1/|d + h| from the Coulomb three-term recurrence.
#pragma once
#include "layout.h"
#include "wave.h"

namespace gtap {
namespace fmm {

constexpr int kP = 6;                                          // expansion order
constexpr int kNc = (kP + 1) * (kP + 2) * (kP + 3) / 6;        // 84 coefficients
constexpr int kBits = 21;                                      // tree depth limit
constexpr int kE = 7;                                          // root half-width 2^7
constexpr int kGrid = kBits - 1 - kE;                          // 2^13 grid units per unit length
constexpr int kCellInts = 8;                                   // level ax ay az begin end child0 nchild

// Number of coefficients of total degree <= d.
constexpr int ncoef(int d) { return (d + 1) * (d + 2) * (d + 3) / 6; }
constexpr int kM2LTerms = 924;  // pairs (a, b) with |a| + |b| <= 6

// Multi-index tables, generated at compile time.  Coefficients are ordered by
// total degree, then by descending x and y exponents.
struct Tables {
  uint8_t e[kNc][3];                     // exponents of coefficient t
  uint8_t idx[kP + 1][kP + 1][kP + 1];   // inverse of e
  uint8_t deg[kNc];
  uint8_t dm1[kNc][3];                   // index of g - e_i (0xFF if g_i == 0)
  uint8_t dm2[kNc][3];                   // index of g - 2 e_i (0xFF if g_i < 2)
  uint16_t m2l_first[kNc + 1];           // terms of target a: [m2l_first[a], m2l_first[a+1])
  uint8_t m2l_b[kM2LTerms];              // source moment index b
  uint8_t m2l_g[kM2LTerms];              // derivative index a + b
  double m2l_c[kM2LTerms];               // C(a + b, a) (-1)^|b|
  double binom[2 * kP + 1][2 * kP + 1];
};

constexpr Tables make_tables() {
  Tables T{};
  for (int n = 0; n <= 2 * kP; ++n) {
    T.binom[n][0] = 1.0;
    for (int k = 1; k <= n; ++k) T.binom[n][k] = T.binom[n - 1][k - 1] + (k < n ? T.binom[n - 1][k] : 0.0);
  }
  int t = 0;
  for (int d = 0; d <= kP; ++d)
    for (int i = d; i >= 0; --i)
      for (int j = d - i; j >= 0; --j) {
        const int k = d - i - j;
        T.e[t][0] = static_cast<uint8_t>(i);
        T.e[t][1] = static_cast<uint8_t>(j);
        T.e[t][2] = static_cast<uint8_t>(k);
        T.idx[i][j][k] = static_cast<uint8_t>(t);
        T.deg[t] = static_cast<uint8_t>(d);
        ++t;
      }
  for (int s = 0; s < kNc; ++s)
    for (int i = 0; i < 3; ++i) {
      int g[3] = {T.e[s][0], T.e[s][1], T.e[s][2]};
      T.dm1[s][i] = 0xFF;
      T.dm2[s][i] = 0xFF;
      if (g[i] >= 1) {
        g[i] -= 1;
        T.dm1[s][i] = T.idx[g[0]][g[1]][g[2]];
        if (g[i] >= 1) {
          g[i] -= 1;
          T.dm2[s][i] = T.idx[g[0]][g[1]][g[2]];
        }
      }
    }
  int m = 0;
  for (int a = 0; a < kNc; ++a) {
    T.m2l_first[a] = static_cast<uint16_t>(m);
    const int da = T.deg[a];
    for (int b = 0; b < ncoef(kP - da); ++b) {
      const int g0 = T.e[a][0] + T.e[b][0], g1 = T.e[a][1] + T.e[b][1], g2 = T.e[a][2] + T.e[b][2];
      T.m2l_b[m] = static_cast<uint8_t>(b);
      T.m2l_g[m] = T.idx[g0][g1][g2];
      const double c = T.binom[g0][T.e[a][0]] * T.binom[g1][T.e[a][1]] * T.binom[g2][T.e[a][2]];
      T.m2l_c[m] = (T.deg[b] & 1) ? -c : c;
      ++m;
    }
  }
  T.m2l_first[kNc] = static_cast<uint16_t>(m);
  return T;
}

__constant__ const Tables kTab = make_tables();
static_assert(make_tables().m2l_first[kNc] == kM2LTerms, "M2L term count");

// Per-job device descriptor of an FMM traversal.
struct FmmDesc {
  const int32_t *cell;     // [ncells][kCellInts]
  const double *Q;         // [ncells][kNc] multipole moments
  double *L;               // [ncells][kNc] local coefficients (accumulated)
  const double *px, *py, *pz, *pq;  // points in sorted order
  double *phi;             // potentials in sorted order (accumulated)
  int64_t ta, tb;          // MAC theta = ta / tb
  uint64_t m2l_pairs, p2p_pairs, m2l_hash, p2p_hash, p2p_inter, coincident;
  // interaction lists (list-building traversals): (target << 32 | source)
  // pairs, appended at m2l_n / p2p_n, which keep counting past the capacity
  uint64_t *m2l_list, *p2p_list;
  uint64_t m2l_cap, p2p_cap;
  uint64_t m2l_n, p2p_n;
  uint32_t ncells;         // a list slot holding target ncells is a gap (see list chunks)
  uint32_t pad_;
};

GTAP_DEV double cell_centre(int32_t anchor, int32_t level) {
  const int64_t w = static_cast<int64_t>(1) << (kBits - level);
  const int64_t c2 = 2 * static_cast<int64_t>(anchor) + w;
  return -static_cast<double>(1 << kE) + static_cast<double>(c2) * (1.0 / static_cast<double>(1 << (kGrid + 1)));
}

GTAP_DEV bool mac_accept(const int32_t *A, const int32_t *B, int64_t ta, int64_t tb) {
  const int64_t wa = static_cast<int64_t>(1) << (kBits - A[0]), wb = static_cast<int64_t>(1) << (kBits - B[0]);
  const int64_t dx = (2 * static_cast<int64_t>(A[1]) + wa) - (2 * static_cast<int64_t>(B[1]) + wb);
  const int64_t dy = (2 * static_cast<int64_t>(A[2]) + wa) - (2 * static_cast<int64_t>(B[2]) + wb);
  const int64_t dz = (2 * static_cast<int64_t>(A[3]) + wa) - (2 * static_cast<int64_t>(B[3]) + wb);
  const __int128 lhs = static_cast<__int128>(3 * tb * tb) * static_cast<__int128>((wa + wb) * (wa + wb));
  const __int128 rhs = static_cast<__int128>(ta * ta) * static_cast<__int128>(dx * dx + dy * dy + dz * dz);
  return lhs < rhs;
}

GTAP_DEV uint64_t pair_hash(uint32_t a, uint32_t b) {
  uint64_t z = (static_cast<uint64_t>(a) << 32) | b;
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ---- tree construction ------------------------------------------------------
GTAP_DEV uint64_t spread3(uint64_t v) {
  v &= 0x1FFFFFull;
  v = (v | (v << 32)) & 0x1F00000000FFFFull;
  v = (v | (v << 16)) & 0x1F0000FF0000FFull;
  v = (v | (v << 8)) & 0x100F00F00F00F00Full;
  v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

GTAP_DEV int64_t grid_coord(double x) {
  const double shifted = __dadd_rn(x, static_cast<double>(1 << kE));
  return static_cast<int64_t>(floor(__dmul_rn(shifted, static_cast<double>(1 << kGrid))));
}

__global__ void k_keys(int32_t n, const double *x, const double *y, const double *z, uint64_t *keys,
                       int32_t *idx, int32_t *bad) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t gx = grid_coord(x[i]), gy = grid_coord(y[i]), gz = grid_coord(z[i]);
  const int64_t lim = static_cast<int64_t>(1) << kBits;
  if (gx < 0 || gy < 0 || gz < 0 || gx >= lim || gy >= lim || gz >= lim) {
    atomicAdd(bad, 1);
    keys[i] = 0;
  } else {
    keys[i] = (spread3(static_cast<uint64_t>(gx)) << 2) | (spread3(static_cast<uint64_t>(gy)) << 1) |
              spread3(static_cast<uint64_t>(gz));
  }
  idx[i] = i;
}

__global__ void k_gather(int32_t n, const int32_t *perm, const double *x, const double *y, const double *z,
                         const double *q, double *px, double *py, double *pz, double *pq, double *phi) {
  const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int32_t i = perm[k];
  px[k] = x[i];
  py[k] = y[i];
  pz[k] = z[i];
  pq[k] = q[i];
  phi[k] = 0.0;
}

__global__ void k_root(int32_t *cell, int32_t *parent, int32_t n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int32_t r[kCellInts] = {0, 0, 0, 0, 0, n, 0, 0};
    for (int i = 0; i < kCellInts; ++i) cell[i] = r[i];
    parent[0] = -1;
  }
}

// Cells [lo, hi) of one level: octant boundaries of each splitting cell by
// binary search in its sorted key range, and the number of non-empty children.
__global__ void k_level_count(int32_t *cell, int32_t lo, int32_t hi, const uint64_t *keys, int32_t leaf_max,
                              int32_t *nch, int32_t *bnd) {
  const int32_t c = lo + static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
  if (c >= hi) return;
  const int32_t *C = cell + static_cast<size_t>(c) * kCellInts;
  const int32_t L = C[0], b = C[4], e = C[5];
  int32_t *B = bnd + static_cast<size_t>(c - lo) * 9;
  int32_t cnt = 0;
  if (e - b > leaf_max && L < kBits) {
    const int shift = 3 * (kBits - 1 - L);
    B[0] = b;
    for (int oct = 1; oct < 8; ++oct) {
      int32_t l = B[oct - 1], r = e;  // first position whose octant digit >= oct
      while (l < r) {
        const int32_t m = l + (r - l) / 2;
        if (static_cast<int>((keys[m] >> shift) & 7u) < oct) l = m + 1;
        else r = m;
      }
      B[oct] = l;
    }
    B[8] = e;
    for (int oct = 0; oct < 8; ++oct) cnt += (B[oct + 1] > B[oct]) ? 1 : 0;
  }
  nch[c - lo] = cnt;
}

// Exclusive scan of nch[0, m) in one workgroup of 1024 threads; *total gets the sum.
__global__ __launch_bounds__(1024) void k_scan(const int32_t *nch, int32_t *off, int32_t m, int32_t *total) {
  __shared__ int32_t part[1024];
  const int32_t t = threadIdx.x;
  const int32_t per = (m + 1023) / 1024;
  const int32_t b = t * per, e = min(m, b + per);
  int32_t s = 0;
  for (int32_t i = b; i < e; ++i) s += nch[i];
  part[t] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const int32_t v = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int32_t run = part[t] - s;
  for (int32_t i = b; i < e; ++i) {
    off[i] = run;
    run += nch[i];
  }
  if (t == 1023) *total = part[1023];
}

__global__ void k_level_write(int32_t *cell, int32_t *parent, int32_t lo, int32_t hi, const int32_t *nch,
                              const int32_t *off, const int32_t *bnd) {
  const int32_t c = lo + static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
  if (c >= hi) return;
  int32_t *C = cell + static_cast<size_t>(c) * kCellInts;
  const int32_t k = nch[c - lo];
  const int32_t first = hi + off[c - lo];
  C[6] = k ? first : 0;
  C[7] = k;
  if (!k) return;
  const int32_t *B = bnd + static_cast<size_t>(c - lo) * 9;
  const int32_t L = C[0], half = 1 << (kBits - 1 - L);
  int32_t w = first;
  for (int oct = 0; oct < 8; ++oct) {
    if (B[oct + 1] == B[oct]) continue;
    int32_t *D = cell + static_cast<size_t>(w) * kCellInts;
    D[0] = L + 1;
    D[1] = C[1] + ((oct >> 2) & 1) * half;
    D[2] = C[2] + ((oct >> 1) & 1) * half;
    D[3] = C[3] + (oct & 1) * half;
    D[4] = B[oct];
    D[5] = B[oct + 1];
    D[6] = 0;
    D[7] = 0;
    parent[w] = c;
    ++w;
  }
}

// ---- upward pass ----------------------------------------------------------------
GTAP_DEV void powers(double v, double *pw) {
  pw[0] = 1.0;
#pragma unroll
  for (int i = 1; i <= kP; ++i) pw[i] = pw[i - 1] * v;
}

// P2M for the leaves among cells [lo, hi): one workgroup of 128 per cell,
// thread t < 84 owns moment t; the leaf's points are staged through LDS.
__global__ __launch_bounds__(128) void k_p2m(const int32_t *cell, int32_t lo, int32_t hi, const double *px,
                                             const double *py, const double *pz, const double *pq, double *Q) {
  const int32_t c = lo + static_cast<int32_t>(blockIdx.x);
  if (c >= hi) return;
  const int32_t *C = cell + static_cast<size_t>(c) * kCellInts;
  if (C[7] != 0) return;
  __shared__ double sx[128], sy[128], sz[128], sq[128];
  const double cx = cell_centre(C[1], C[0]), cy = cell_centre(C[2], C[0]), cz = cell_centre(C[3], C[0]);
  const int t = threadIdx.x;
  double acc = 0.0;
  const int ex = t < kNc ? kTab.e[t][0] : 0, ey = t < kNc ? kTab.e[t][1] : 0, ez = t < kNc ? kTab.e[t][2] : 0;
  for (int32_t b = C[4]; b < C[5]; b += 128) {
    const int32_t k = b + t;
    if (k < C[5]) {
      sx[t] = px[k] - cx;
      sy[t] = py[k] - cy;
      sz[t] = pz[k] - cz;
      sq[t] = pq[k];
    }
    __syncthreads();
    const int m = min(128, C[5] - b);
    if (t < kNc)
      for (int j = 0; j < m; ++j) {
        double v = sq[j];
        for (int i = 0; i < ex; ++i) v *= sx[j];
        for (int i = 0; i < ey; ++i) v *= sy[j];
        for (int i = 0; i < ez; ++i) v *= sz[j];
        acc += v;
      }
    __syncthreads();
  }
  if (t < kNc) Q[static_cast<size_t>(c) * kNc + t] = acc;
}

// M2M for the internal cells among [lo, hi) (children already final).
__global__ __launch_bounds__(128) void k_m2m(const int32_t *cell, int32_t lo, int32_t hi, double *Q) {
  const int32_t c = lo + static_cast<int32_t>(blockIdx.x);
  if (c >= hi) return;
  const int32_t *C = cell + static_cast<size_t>(c) * kCellInts;
  if (C[7] == 0) return;
  const int t = threadIdx.x;
  if (t >= kNc) return;
  const double cx = cell_centre(C[1], C[0]), cy = cell_centre(C[2], C[0]), cz = cell_centre(C[3], C[0]);
  const int b0 = kTab.e[t][0], b1 = kTab.e[t][1], b2 = kTab.e[t][2];
  double acc = 0.0;
  for (int32_t k = 0; k < C[7]; ++k) {
    const int32_t ch = C[6] + k;
    const int32_t *D = cell + static_cast<size_t>(ch) * kCellInts;
    double sx[kP + 1], sy[kP + 1], sz[kP + 1];
    powers(cell_centre(D[1], D[0]) - cx, sx);
    powers(cell_centre(D[2], D[0]) - cy, sy);
    powers(cell_centre(D[3], D[0]) - cz, sz);
    const double *Qc = Q + static_cast<size_t>(ch) * kNc;
    for (int i = 0; i <= b0; ++i)
      for (int j = 0; j <= b1; ++j)
        for (int l = 0; l <= b2; ++l)
          acc += kTab.binom[b0][i] * kTab.binom[b1][j] * kTab.binom[b2][l] * Qc[kTab.idx[i][j][l]] *
                 sx[b0 - i] * sy[b1 - j] * sz[b2 - l];
  }
  Q[static_cast<size_t>(c) * kNc + t] = acc;
}

// ---- downward pass --------------------------------------------------------------
// L2L into the cells [lo, hi) from their parents (parents already final).
__global__ __launch_bounds__(128) void k_l2l(const int32_t *cell, const int32_t *parent, int32_t lo, int32_t hi,
                                             double *L) {
  const int32_t c = lo + static_cast<int32_t>(blockIdx.x);
  if (c >= hi) return;
  const int t = threadIdx.x;
  if (t >= kNc) return;
  const int32_t pc = parent[c];
  const int32_t *C = cell + static_cast<size_t>(c) * kCellInts;
  const int32_t *P = cell + static_cast<size_t>(pc) * kCellInts;
  double sx[kP + 1], sy[kP + 1], sz[kP + 1];
  powers(cell_centre(C[1], C[0]) - cell_centre(P[1], P[0]), sx);
  powers(cell_centre(C[2], C[0]) - cell_centre(P[2], P[0]), sy);
  powers(cell_centre(C[3], C[0]) - cell_centre(P[3], P[0]), sz);
  const double *Lp = L + static_cast<size_t>(pc) * kNc;
  const int v0 = kTab.e[t][0], v1 = kTab.e[t][1], v2 = kTab.e[t][2];
  double acc = 0.0;
  for (int u = 0; u < kNc; ++u) {
    const int a0 = kTab.e[u][0], a1 = kTab.e[u][1], a2 = kTab.e[u][2];
    if (a0 < v0 || a1 < v1 || a2 < v2) continue;
    acc += kTab.binom[a0][v0] * kTab.binom[a1][v1] * kTab.binom[a2][v2] * Lp[u] * sx[a0 - v0] * sy[a1 - v1] *
           sz[a2 - v2];
  }
  L[static_cast<size_t>(c) * kNc + t] += acc;
}

// L2P for the leaves among [lo, hi): thread per point.
__global__ __launch_bounds__(128) void k_l2p(const int32_t *cell, int32_t lo, int32_t hi, const double *L,
                                             const double *px, const double *py, const double *pz, double *phi) {
  const int32_t c = lo + static_cast<int32_t>(blockIdx.x);
  if (c >= hi) return;
  const int32_t *C = cell + static_cast<size_t>(c) * kCellInts;
  if (C[7] != 0) return;
  __shared__ double sL[kNc];
  if (threadIdx.x < kNc) sL[threadIdx.x] = L[static_cast<size_t>(c) * kNc + threadIdx.x];
  __syncthreads();
  const double cx = cell_centre(C[1], C[0]), cy = cell_centre(C[2], C[0]), cz = cell_centre(C[3], C[0]);
  for (int32_t k = C[4] + static_cast<int32_t>(threadIdx.x); k < C[5]; k += blockDim.x) {
    double sx[kP + 1], sy[kP + 1], sz[kP + 1];
    powers(px[k] - cx, sx);
    powers(py[k] - cy, sy);
    powers(pz[k] - cz, sz);
    double acc = 0.0;
    for (int u = 0; u < kNc; ++u) acc += sL[u] * sx[kTab.e[u][0]] * sy[kTab.e[u][1]] * sz[kTab.e[u][2]];
    phi[k] += acc;
  }
}

__global__ void k_scatter(int32_t n, const int32_t *perm, const double *phi_sorted, double *phi) {
  const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) phi[perm[k]] = phi_sorted[k];
}

}  // namespace fmm
}  // namespace gtap
