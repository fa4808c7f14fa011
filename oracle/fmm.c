/*
 * fmm.c -- plain, sequential CPU oracle of the 3D Laplace FMM pipeline with a
 * dual-tree traversal (GTaP Sec. 6.4.1, "FMM Dual-Tree Traversal": adaptive
 * octree, upward pass, DTT over cell pairs with a multipole acceptance
 * criterion, M2L, P2P and L2P).
 *
 * TEST INFRASTRUCTURE. Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  The HIP runtime never
 * calls it and shares no code, header, table or constant generator with it.
 *
 * The paper names the phases only; every detail below is a stated reading:
 *  - Root cube [-2^E, 2^E)^3 with E = 7.  Integer grid coordinate of x:
 *    floor((x + 2^E) * 2^(20-E)) in [0, 2^21) (one rounded add, then an exact
 *    scaling).  63-bit Morton key, bit 3k+2 from x, 3k+1 from y, 3k from z.
 *    Points are ordered by (key, original index).
 *  - A cell splits iff it holds more than leaf_max points and its level is
 *    below 21.  Only non-empty children exist.  Cells are numbered
 *    breadth-first, level by level, Morton order within a level; the
 *    children of a cell are contiguous.
 *  - Cell geometry in grid units: anchor a, width w = 2^(21-level); doubled
 *    centre C2 = 2a + w; physical centre -2^E + C2 * 2^(E-21).
 *  - MAC theta = ta/tb with R the half cube diagonal, exact in integers:
 *    accept (A,B) iff 3 tb^2 (w_A + w_B)^2 < ta^2 |C2_A - C2_B|^2.
 *  - DTT from (root, root): accept -> M2L(A <- B); both leaves -> P2P(A <- B);
 *    else split the wider cell; on equal widths split A unless A is a leaf;
 *    a leaf is never split (the other cell is).
 *  - Expansions: Cartesian Taylor series of 1/|x - y| truncated at total
 *    degree p in (x - c_A, y - c_B).  Multipole moments
 *    Q_b = sum_j q_j (y_j - c_B)^b; local coefficients
 *    L_a = sum_{|b| <= p-|a|} C(a+b, a) (-1)^|b| T_{a+b}(d) Q_b with
 *    d = c_A - c_B and T_g the Taylor coefficients of 1/|d + h| in h;
 *    potential sum_a L_a (x - c_A)^a.  M2M and L2L are the exact binomial
 *    re-centrings of these polynomials.
 *  - Kernel 1/r without 1/(4 pi); j == i is skipped; distinct points at the
 *    same position are skipped and counted.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_FMM_E 7
#define ORC_FMM_BITS 21
#define ORC_FMM_GRID (ORC_FMM_BITS - 1 - ORC_FMM_E) /* grid units per length unit: 2^13 */
#define ORC_PMAX 10
#define ORC_NCOEF_MAX 286 /* (PMAX+1)(PMAX+2)(PMAX+3)/6 */

typedef struct {
    int32_t level;
    int32_t ax, ay, az;      /* anchor, grid units */
    int32_t begin, end;      /* range of sorted points */
    int32_t child0, nchild;  /* children are cells child0 .. child0+nchild-1 */
    int32_t parent;
} orc_cell;

typedef struct {
    int64_t n_cells, n_leaves, max_level;
    int64_t m2l_pairs, p2p_pairs;
    uint64_t m2l_hash, p2p_hash;  /* wrapping sums of mix64(A << 32 | B) */
    int64_t p2p_interactions, coincident;
} orc_fmm_stats;

/* ---- multi-indices ------------------------------------------------------ */
/* Pascal's triangle up to row 2 PMAX. */
static double binom_t[2 * ORC_PMAX + 1][2 * ORC_PMAX + 1];

static void binom_init(void)
{
    for (int n = 0; n <= 2 * ORC_PMAX; n++) {
        binom_t[n][0] = 1.0;
        for (int k = 1; k <= n; k++) binom_t[n][k] = binom_t[n - 1][k - 1] + (k < n ? binom_t[n - 1][k] : 0.0);
    }
}

static double binom(int n, int k) { return binom_t[n][k]; }

typedef struct {
    int p, n;
    int a[ORC_NCOEF_MAX][3];
    int idx[ORC_PMAX + 1][ORC_PMAX + 1][ORC_PMAX + 1];
} mindex;

static void mindex_init(mindex *m, int p)
{
    binom_init();
    m->p = p;
    m->n = 0;
    for (int deg = 0; deg <= p; deg++)
        for (int i = deg; i >= 0; i--)
            for (int j = deg - i; j >= 0; j--) {
                int k = deg - i - j;
                m->a[m->n][0] = i;
                m->a[m->n][1] = j;
                m->a[m->n][2] = k;
                m->idx[i][j][k] = m->n++;
            }
}


/* Taylor coefficients T_g(d) of 1/|d + h| in h for |g| <= p, from the
 * three-term recurrence of the Coulomb kernel's Cartesian Taylor
 * coefficients (as used by Cartesian treecodes, e.g. Duan and Krasny 2001):
 *   |g| |d|^2 T_g = -(2|g| - 1) sum_i d_i T_{g - e_i} - (|g| - 1) sum_i T_{g - 2 e_i}. */
static void taylor_coulomb(const mindex *m, const double d[3], double *T)
{
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    T[0] = 1.0 / sqrt(r2);
    for (int t = 1; t < m->n; t++) {
        const int *g = m->a[t];
        int deg = g[0] + g[1] + g[2];
        double s1 = 0.0, s2 = 0.0;
        for (int i = 0; i < 3; i++) {
            int h[3] = {g[0], g[1], g[2]};
            if (h[i] >= 1) {
                h[i] -= 1;
                s1 += d[i] * T[m->idx[h[0]][h[1]][h[2]]];
                if (h[i] >= 1) {
                    h[i] -= 1;
                    s2 += T[m->idx[h[0]][h[1]][h[2]]];
                }
            }
        }
        T[t] = -((2.0 * deg - 1.0) * s1 + (deg - 1.0) * s2) / (deg * r2);
    }
}

static void powers(double v, int p, double *pw)
{
    pw[0] = 1.0;
    for (int i = 1; i <= p; i++) pw[i] = pw[i - 1] * v;
}

/* ---- tree ------------------------------------------------------------------ */
typedef struct {
    uint64_t key;
    int64_t idx;
} keyed;

static int cmp_keyed(const void *x, const void *y)
{
    const keyed *a = (const keyed *)x, *b = (const keyed *)y;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

static uint64_t spread3(uint64_t v)
{
    uint64_t r = 0;
    for (int b = 0; b < ORC_FMM_BITS; b++) r |= ((v >> b) & 1ull) << (3 * b);
    return r;
}

static int64_t grid_coord(double x)
{
    const double shift = (double)(1 << ORC_FMM_E);
    const double scale = (double)(1 << ORC_FMM_GRID);
    return (int64_t)floor((x + shift) * scale);
}

static double cell_centre(int32_t anchor, int level)
{
    int64_t w = (int64_t)1 << (ORC_FMM_BITS - level);
    int64_t c2 = 2 * (int64_t)anchor + w;
    return -(double)(1 << ORC_FMM_E) + (double)c2 * ldexp(1.0, -(ORC_FMM_GRID + 1));
}

/* Build the octree.  perm[k] = original index of the k-th sorted point.
 * Returns the number of cells, -1 if a point lies outside the root cube, -2 if
 * more than cap cells are needed. */
int64_t orc_fmm_tree(int64_t n, const double *x, const double *y, const double *z, int leaf_max,
                     int32_t *perm, orc_cell *cells, int64_t cap, uint64_t *keys_out)
{
    keyed *kv = (keyed *)malloc(sizeof(keyed) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; i++) {
        int64_t g[3] = {grid_coord(x[i]), grid_coord(y[i]), grid_coord(z[i])};
        for (int c = 0; c < 3; c++)
            if (g[c] < 0 || g[c] >= ((int64_t)1 << ORC_FMM_BITS)) {
                free(kv);
                return -1;
            }
        kv[i].key = (spread3((uint64_t)g[0]) << 2) | (spread3((uint64_t)g[1]) << 1) | spread3((uint64_t)g[2]);
        kv[i].idx = i;
    }
    qsort(kv, (size_t)n, sizeof(keyed), cmp_keyed);
    for (int64_t k = 0; k < n; k++) {
        perm[k] = (int32_t)kv[k].idx;
        if (keys_out) keys_out[k] = kv[k].key;
    }
    if (cap < 1) {
        free(kv);
        return -2;
    }
    int64_t nc = 1;
    cells[0] = (orc_cell){0, 0, 0, 0, 0, (int32_t)n, 0, 0, -1};
    for (int64_t c = 0; c < nc; c++) {  /* cells are visited in creation order: breadth-first */
        orc_cell *C = &cells[c];
        int L = C->level;
        if (C->end - C->begin <= leaf_max || L >= ORC_FMM_BITS) continue;
        int shift = 3 * (ORC_FMM_BITS - 1 - L);
        int32_t half = (int32_t)1 << (ORC_FMM_BITS - 1 - L);
        int32_t k = C->begin;
        C->child0 = (int32_t)nc;
        for (int oct = 0; oct < 8; oct++) {
            int32_t b = k;
            while (k < C->end && (int)((kv[k].key >> shift) & 7u) == oct) k++;
            if (k == b) continue;
            if (nc >= cap) {
                free(kv);
                return -2;
            }
            orc_cell ch;
            ch.level = L + 1;
            ch.ax = C->ax + ((oct >> 2) & 1) * half;
            ch.ay = C->ay + ((oct >> 1) & 1) * half;
            ch.az = C->az + (oct & 1) * half;
            ch.begin = b;
            ch.end = k;
            ch.child0 = 0;
            ch.nchild = 0;
            ch.parent = (int32_t)c;
            cells[nc++] = ch;
            C = &cells[c];
            C->nchild++;
        }
    }
    free(kv);
    return nc;
}

/* ---- traversal ------------------------------------------------------------ */
static uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static int accept_pair(const orc_cell *A, const orc_cell *B, int64_t ta, int64_t tb)
{
    int64_t wa = (int64_t)1 << (ORC_FMM_BITS - A->level), wb = (int64_t)1 << (ORC_FMM_BITS - B->level);
    int64_t dx = (2 * (int64_t)A->ax + wa) - (2 * (int64_t)B->ax + wb);
    int64_t dy = (2 * (int64_t)A->ay + wa) - (2 * (int64_t)B->ay + wb);
    int64_t dz = (2 * (int64_t)A->az + wa) - (2 * (int64_t)B->az + wb);
    __int128 lhs = (__int128)3 * tb * tb * (__int128)((wa + wb) * (wa + wb));
    __int128 rhs = (__int128)ta * ta * (__int128)(dx * dx + dy * dy + dz * dz);
    return lhs < rhs;
}

typedef struct {
    int32_t *m2l, *p2p; /* pairs (A, B) */
    int64_t nm2l, np2p, cap_m2l, cap_p2p;
} pair_lists;

static void push_pair(int32_t **v, int64_t *len, int64_t *cap, int32_t a, int32_t b)
{
    if (*len >= *cap) {
        *cap = *cap ? 2 * *cap : 1024;
        *v = (int32_t *)realloc(*v, sizeof(int32_t) * 2 * (size_t)*cap);
    }
    (*v)[2 * *len] = a;
    (*v)[2 * *len + 1] = b;
    (*len)++;
}

static void dual_tree(const orc_cell *cells, int64_t ta, int64_t tb, pair_lists *pl)
{
    int64_t sn = 0, scap = 1024;
    int32_t *st = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)scap);
    st[0] = 0;
    st[1] = 0;
    sn = 1;
    while (sn > 0) {
        sn--;
        int32_t a = st[2 * sn], b = st[2 * sn + 1];
        const orc_cell *A = &cells[a], *B = &cells[b];
        if (accept_pair(A, B, ta, tb)) {
            push_pair(&pl->m2l, &pl->nm2l, &pl->cap_m2l, a, b);
            continue;
        }
        int leaf_a = A->nchild == 0, leaf_b = B->nchild == 0;
        if (leaf_a && leaf_b) {
            push_pair(&pl->p2p, &pl->np2p, &pl->cap_p2p, a, b);
            continue;
        }
        int split_a;
        if (A->level < B->level) split_a = 1;       /* A is wider */
        else if (A->level > B->level) split_a = 0;  /* B is wider */
        else split_a = !leaf_a;
        if (split_a && leaf_a) split_a = 0;
        if (!split_a && leaf_b) split_a = 1;
        const orc_cell *S = split_a ? A : B;
        for (int32_t c = 0; c < S->nchild; c++) {
            int32_t ch = S->child0 + c;
            if (sn >= scap) {
                scap *= 2;
                st = (int32_t *)realloc(st, sizeof(int32_t) * 2 * (size_t)scap);
            }
            st[2 * sn] = split_a ? ch : a;
            st[2 * sn + 1] = split_a ? b : ch;
            sn++;
        }
    }
    free(st);
}

/* ---- expansions ----------------------------------------------------------- */
static void p2m(const mindex *m, const orc_cell *C, const int32_t *perm, const double *x, const double *y,
                const double *z, const double *q, double *Q)
{
    double c[3] = {cell_centre(C->ax, C->level), cell_centre(C->ay, C->level), cell_centre(C->az, C->level)};
    double px[ORC_PMAX + 1], py[ORC_PMAX + 1], pz[ORC_PMAX + 1];
    for (int t = 0; t < m->n; t++) Q[t] = 0.0;
    for (int32_t k = C->begin; k < C->end; k++) {
        int32_t j = perm[k];
        powers(x[j] - c[0], m->p, px);
        powers(y[j] - c[1], m->p, py);
        powers(z[j] - c[2], m->p, pz);
        for (int t = 0; t < m->n; t++) Q[t] += q[j] * px[m->a[t][0]] * py[m->a[t][1]] * pz[m->a[t][2]];
    }
}

/* Q_parent += moments of the child re-centred: (y - c) = (y - c') + s. */
static void m2m(const mindex *m, const double *Qc, const double s[3], double *Qp)
{
    double ps[3][ORC_PMAX + 1];
    for (int i = 0; i < 3; i++) powers(s[i], m->p, ps[i]);
    for (int t = 0; t < m->n; t++) {
        const int *b = m->a[t];
        double acc = 0.0;
        for (int i = 0; i <= b[0]; i++)
            for (int j = 0; j <= b[1]; j++)
                for (int k = 0; k <= b[2]; k++)
                    acc += binom(b[0], i) * binom(b[1], j) * binom(b[2], k) * Qc[m->idx[i][j][k]] *
                           ps[0][b[0] - i] * ps[1][b[1] - j] * ps[2][b[2] - k];
        Qp[t] += acc;
    }
}

static void m2l(const mindex *m, const double *QB, const double d[3], double *LA)
{
    double T[ORC_NCOEF_MAX];
    taylor_coulomb(m, d, T);
    for (int t = 0; t < m->n; t++) {
        const int *a = m->a[t];
        int da = a[0] + a[1] + a[2];
        double acc = 0.0;
        /* graded order: the b with |b| <= p - |a| are the first ones */
        const int nb = (m->p - da + 1) * (m->p - da + 2) * (m->p - da + 3) / 6;
        for (int u = 0; u < nb; u++) {
            const int *b = m->a[u];
            int db = b[0] + b[1] + b[2];
            double cf = binom(a[0] + b[0], a[0]) * binom(a[1] + b[1], a[1]) * binom(a[2] + b[2], a[2]);
            double sg = (db & 1) ? -1.0 : 1.0;
            acc += cf * sg * T[m->idx[a[0] + b[0]][a[1] + b[1]][a[2] + b[2]]] * QB[u];
        }
        LA[t] += acc;
    }
}

/* L_child += parent's local polynomial re-centred: (x - c) = (x - c') + s. */
static void l2l(const mindex *m, const double *Lp, const double s[3], double *Lc)
{
    double ps[3][ORC_PMAX + 1];
    for (int i = 0; i < 3; i++) powers(s[i], m->p, ps[i]);
    for (int t = 0; t < m->n; t++) {
        const int *v = m->a[t];
        double acc = 0.0;
        for (int u = 0; u < m->n; u++) {
            const int *a = m->a[u];
            if (a[0] < v[0] || a[1] < v[1] || a[2] < v[2]) continue;
            acc += binom(a[0], v[0]) * binom(a[1], v[1]) * binom(a[2], v[2]) * Lp[u] * ps[0][a[0] - v[0]] *
                   ps[1][a[1] - v[1]] * ps[2][a[2] - v[2]];
        }
        Lc[t] += acc;
    }
}

static double l2p(const mindex *m, const double *L, const double r[3])
{
    double px[ORC_PMAX + 1], py[ORC_PMAX + 1], pz[ORC_PMAX + 1];
    powers(r[0], m->p, px);
    powers(r[1], m->p, py);
    powers(r[2], m->p, pz);
    double acc = 0.0;
    for (int t = 0; t < m->n; t++) acc += L[t] * px[m->a[t][0]] * py[m->a[t][1]] * pz[m->a[t][2]];
    return acc;
}

static double p2p_one(int32_t i, const orc_cell *B, const int32_t *perm, const double *x, const double *y,
                      const double *z, const double *q, int64_t *inter, int64_t *coinc)
{
    double acc = 0.0;
    for (int32_t k = B->begin; k < B->end; k++) {
        int32_t j = perm[k];
        if (j == i) continue;
        double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
        double r2 = dx * dx + dy * dy + dz * dz;
        (*inter)++;
        if (r2 == 0.0) {
            (*coinc)++;
            continue;
        }
        acc += q[j] / sqrt(r2);
    }
    return acc;
}

static void cell_centre3(const orc_cell *C, double c[3])
{
    c[0] = cell_centre(C->ax, C->level);
    c[1] = cell_centre(C->ay, C->level);
    c[2] = cell_centre(C->az, C->level);
}

/*
 * The FMM pipeline.  targets == NULL: phi[i] for every point, by the passes
 * in order (P2M, M2M, DTT, M2L into the target cell, L2L, L2P, P2P).
 * Otherwise phi[t] for the listed targets only, each as P2P over its leaf's
 * P2P partners plus, for every M2L pair whose target cell contains it, that
 * pair's local expansion evaluated at the point (equal to the full passes up
 * to rounding, as L2L is exact).
 * m2l_out / p2p_out (optional, 2 * list_cap int32 each) receive the pair lists.
 * Returns 0, or -1 (point outside the root cube), -2 (allocation), -3 (bad p).
 */
int orc_fmm(int64_t n, const double *x, const double *y, const double *z, const double *q, int p, int64_t ta,
            int64_t tb, int leaf_max, const int64_t *targets, int64_t ntargets, double *phi, orc_fmm_stats *st,
            int32_t *m2l_out, int32_t *p2p_out, int64_t list_cap)
{
    if (p < 0 || p > ORC_PMAX) return -3;
    memset(st, 0, sizeof(*st));
    mindex *m = (mindex *)malloc(sizeof(mindex));
    mindex_init(m, p);
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t cap = 2 * (n > 0 ? n : 1) + 64;
    orc_cell *cells = (orc_cell *)malloc(sizeof(orc_cell) * (size_t)cap);
    int64_t nc = orc_fmm_tree(n, x, y, z, leaf_max, perm, cells, cap, NULL);
    if (nc < 0) {
        free(m);
        free(perm);
        free(cells);
        return nc == -1 ? -1 : -2;
    }
    st->n_cells = nc;
    for (int64_t c = 0; c < nc; c++) {
        if (cells[c].nchild == 0) st->n_leaves++;
        if (cells[c].level > st->max_level) st->max_level = cells[c].level;
    }
    const int nco = m->n;
    double *Q = (double *)calloc((size_t)(nc * nco), sizeof(double));
    /* upward pass: P2M at leaves, M2M from the deepest cells up */
    for (int64_t c = nc - 1; c >= 0; c--) {
        const orc_cell *C = &cells[c];
        if (C->nchild == 0) {
            p2m(m, C, perm, x, y, z, q, Q + c * nco);
        } else {
            double cp[3];
            cell_centre3(C, cp);
            for (int32_t k = 0; k < C->nchild; k++) {
                double cc[3], s[3];
                cell_centre3(&cells[C->child0 + k], cc);
                for (int i = 0; i < 3; i++) s[i] = cc[i] - cp[i];
                m2m(m, Q + (int64_t)(C->child0 + k) * nco, s, Q + c * nco);
            }
        }
    }
    /* dual-tree traversal */
    pair_lists pl;
    memset(&pl, 0, sizeof(pl));
    dual_tree(cells, ta, tb, &pl);
    st->m2l_pairs = pl.nm2l;
    st->p2p_pairs = pl.np2p;
    for (int64_t k = 0; k < pl.nm2l; k++)
        st->m2l_hash += mix64(((uint64_t)(uint32_t)pl.m2l[2 * k] << 32) | (uint32_t)pl.m2l[2 * k + 1]);
    for (int64_t k = 0; k < pl.np2p; k++)
        st->p2p_hash += mix64(((uint64_t)(uint32_t)pl.p2p[2 * k] << 32) | (uint32_t)pl.p2p[2 * k + 1]);
    if (m2l_out)
        memcpy(m2l_out, pl.m2l, sizeof(int32_t) * 2 * (size_t)(pl.nm2l < list_cap ? pl.nm2l : list_cap));
    if (p2p_out)
        memcpy(p2p_out, pl.p2p, sizeof(int32_t) * 2 * (size_t)(pl.np2p < list_cap ? pl.np2p : list_cap));

    if (targets == NULL) {
        double *L = (double *)calloc((size_t)(nc * nco), sizeof(double));
        for (int64_t k = 0; k < pl.nm2l; k++) {
            const orc_cell *A = &cells[pl.m2l[2 * k]], *B = &cells[pl.m2l[2 * k + 1]];
            double ca[3], cb[3], d[3];
            cell_centre3(A, ca);
            cell_centre3(B, cb);
            for (int i = 0; i < 3; i++) d[i] = ca[i] - cb[i];
            m2l(m, Q + (int64_t)pl.m2l[2 * k + 1] * nco, d, L + (int64_t)pl.m2l[2 * k] * nco);
        }
        /* downward pass: L2L from the root down, L2P at leaves */
        for (int64_t c = 0; c < nc; c++) {
            const orc_cell *C = &cells[c];
            double cp[3];
            cell_centre3(C, cp);
            for (int32_t k = 0; k < C->nchild; k++) {
                double cc[3], s[3];
                cell_centre3(&cells[C->child0 + k], cc);
                for (int i = 0; i < 3; i++) s[i] = cc[i] - cp[i];
                l2l(m, L + c * nco, s, L + (int64_t)(C->child0 + k) * nco);
            }
        }
        for (int64_t i = 0; i < n; i++) phi[i] = 0.0;
        for (int64_t c = 0; c < nc; c++) {
            const orc_cell *C = &cells[c];
            if (C->nchild) continue;
            double cp[3];
            cell_centre3(C, cp);
            for (int32_t k = C->begin; k < C->end; k++) {
                int32_t i = perm[k];
                double r[3] = {x[i] - cp[0], y[i] - cp[1], z[i] - cp[2]};
                phi[i] += l2p(m, L + c * nco, r);
            }
        }
        for (int64_t k = 0; k < pl.np2p; k++) {
            const orc_cell *A = &cells[pl.p2p[2 * k]], *B = &cells[pl.p2p[2 * k + 1]];
            for (int32_t t = A->begin; t < A->end; t++) {
                int32_t i = perm[t];
                phi[i] += p2p_one(i, B, perm, x, y, z, q, &st->p2p_interactions, &st->coincident);
            }
        }
        free(L);
    } else {
        /* sorted position of every point, and the leaf holding it */
        int32_t *rank = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        int32_t *leaf_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        for (int64_t k = 0; k < n; k++) rank[perm[k]] = (int32_t)k;
        for (int64_t c = 0; c < nc; c++)
            if (cells[c].nchild == 0)
                for (int32_t k = cells[c].begin; k < cells[c].end; k++) leaf_of[k] = (int32_t)c;
        /* pair lists grouped by target cell */
        int64_t *m_off = (int64_t *)calloc((size_t)(nc + 1), sizeof(int64_t));
        int64_t *p_off = (int64_t *)calloc((size_t)(nc + 1), sizeof(int64_t));
        for (int64_t k = 0; k < pl.nm2l; k++) m_off[pl.m2l[2 * k] + 1]++;
        for (int64_t k = 0; k < pl.np2p; k++) p_off[pl.p2p[2 * k] + 1]++;
        for (int64_t c = 0; c < nc; c++) {
            m_off[c + 1] += m_off[c];
            p_off[c + 1] += p_off[c];
        }
        int32_t *m_src = (int32_t *)malloc(sizeof(int32_t) * (size_t)(pl.nm2l + 1));
        int32_t *p_src = (int32_t *)malloc(sizeof(int32_t) * (size_t)(pl.np2p + 1));
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nc + 1));
        memcpy(fill, m_off, sizeof(int64_t) * (size_t)nc);
        for (int64_t k = 0; k < pl.nm2l; k++) m_src[fill[pl.m2l[2 * k]]++] = pl.m2l[2 * k + 1];
        memcpy(fill, p_off, sizeof(int64_t) * (size_t)nc);
        for (int64_t k = 0; k < pl.np2p; k++) p_src[fill[pl.p2p[2 * k]]++] = pl.p2p[2 * k + 1];
        free(fill);
        double *Lp = (double *)malloc(sizeof(double) * (size_t)nco);
        for (int64_t t = 0; t < ntargets; t++) {
            int64_t i = targets[t];
            int32_t lf = leaf_of[rank[i]];
            double acc = 0.0;
            /* M2L pairs whose target cell is the leaf of i or one of its ancestors */
            for (int32_t a = lf; a >= 0; a = cells[a].parent) {
                const orc_cell *A = &cells[a];
                double ca[3];
                cell_centre3(A, ca);
                double r[3] = {x[i] - ca[0], y[i] - ca[1], z[i] - ca[2]};
                for (int64_t k = m_off[a]; k < m_off[a + 1]; k++) {
                    double cb[3], d[3];
                    cell_centre3(&cells[m_src[k]], cb);
                    for (int u = 0; u < 3; u++) d[u] = ca[u] - cb[u];
                    for (int u = 0; u < nco; u++) Lp[u] = 0.0;
                    m2l(m, Q + (int64_t)m_src[k] * nco, d, Lp);
                    acc += l2p(m, Lp, r);
                }
            }
            for (int64_t k = p_off[lf]; k < p_off[lf + 1]; k++)
                acc += p2p_one((int32_t)i, &cells[p_src[k]], perm, x, y, z, q, &st->p2p_interactions,
                               &st->coincident);
            phi[t] = acc;
        }
        free(m_off);
        free(p_off);
        free(m_src);
        free(p_src);
        free(Lp);
        free(rank);
        free(leaf_of);
    }
    free(pl.m2l);
    free(pl.p2p);
    free(Q);
    free(m);
    free(perm);
    free(cells);
    return 0;
}

/* Direct summation at the listed targets: sum over j != i of q_j / |x_i - x_j|
 * (coincident distinct points skipped). */
void orc_direct(int64_t n, const double *x, const double *y, const double *z, const double *q,
                const int64_t *targets, int64_t ntargets, double *phi)
{
    for (int64_t t = 0; t < ntargets; t++) {
        int64_t i = targets[t];
        double acc = 0.0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            acc += q[j] / sqrt(r2);
        }
        phi[t] = acc;
    }
}
