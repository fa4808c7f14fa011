/*
 * synth.c -- seeded synthetic input generators (host side, plain C).
 *
 * These produce the inputs both the HIP runtime and the CPU oracle consume:
 * power-law graphs and their acyclic orientation.  Nothing here computes any
 * part of a workload's result; the k-clique count of a graph does not depend
 * on which acyclic orientation it is given.
 *
 * Random numbers come from splitmix64 (Steele, Lea, Flood, OOPSLA 2014),
 * written from its published definition; draw e of stream `seed` is
 * mix64(seed + (e+1) * gamma).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SYN_GAMMA 0x9E3779B97F4A7C15ull

static uint64_t syn_mix64(uint64_t z)
{
    z += SYN_GAMMA;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t syn_draw(uint64_t seed, uint64_t e) { return syn_mix64(seed + (e + 1) * SYN_GAMMA); }

static uint64_t mulhi64(uint64_t a, uint64_t b)
{
    return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) >> 64);
}

/* LSD radix sort of 64-bit keys, 16 bits per pass. */
static void radix_sort_u64(uint64_t *a, int64_t n, uint64_t *tmp)
{
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * 65536);
    uint64_t *src = a, *dst = tmp;
    for (int pass = 0; pass < 4; pass++) {
        int sh = pass * 16;
        memset(cnt, 0, sizeof(int64_t) * 65536);
        for (int64_t i = 0; i < n; i++) cnt[(src[i] >> sh) & 0xFFFF]++;
        int64_t s = 0;
        for (int b = 0; b < 65536; b++) {
            int64_t c = cnt[b];
            cnt[b] = s;
            s += c;
        }
        for (int64_t i = 0; i < n; i++) dst[cnt[(src[i] >> sh) & 0xFFFF]++] = src[i];
        uint64_t *t = src;
        src = dst;
        dst = t;
    }
    /* four passes: result is back in a */
    free(cnt);
}

/*
 * Chung-Lu power-law graph.  Expected-degree weights b_i = (i+1)^(-1/(g-1)),
 * scaled by c so that mean(min(c b_i, cap)) = dbar with cap = cap_frac
 * sqrt(n dbar); weights are quantised to 20 fractional bits and m = round(n
 * dbar / 2) edges are drawn with both endpoints proportional to weight.
 * Self-loops and duplicate edges are dropped.
 *
 * out_keys must hold round(n*dbar/2) entries; it receives the sorted unique
 * undirected edges as (min << 32 | max).  Returns the number of edges, or -1.
 */
int64_t syn_chung_lu(int64_t n, double dbar, double gamma, double cap_frac,
                     uint64_t seed, uint64_t *out_keys, double *out_scale)
{
    if (n < 2 || n > 2000000000 || dbar <= 0 || gamma <= 1.0) return -1;
    double *b = (double *)malloc(sizeof(double) * n);
    for (int64_t i = 0; i < n; i++) b[i] = pow((double)(i + 1), -1.0 / (gamma - 1.0));
    double cap = cap_frac * sqrt((double)n * dbar);
    /* bisection on c: mean(min(c b_i, cap)) is non-decreasing in c */
    double lo = 0.0, hi = 1.0;
    for (;;) {
        double s = 0;
        for (int64_t i = 0; i < n; i++) s += fmin(hi * b[i], cap);
        if (s / n >= dbar || hi > 1e300) break;
        hi *= 2.0;
    }
    for (int it = 0; it < 200; it++) {
        double mid = 0.5 * (lo + hi), s = 0;
        for (int64_t i = 0; i < n; i++) s += fmin(mid * b[i], cap);
        if (s / n < dbar) lo = mid;
        else hi = mid;
    }
    double c = hi;
    if (out_scale) *out_scale = c;
    uint64_t *S = (uint64_t *)malloc(sizeof(uint64_t) * n);
    uint64_t acc = 0;
    for (int64_t i = 0; i < n; i++) {
        double w = fmin(c * b[i], cap);
        acc += (uint64_t)llround(w * 1048576.0);
        S[i] = acc;
    }
    free(b);
    uint64_t tot = acc;
    int64_t m = (int64_t)llround((double)n * dbar / 2.0);
    int64_t k = 0;
    for (int64_t e = 0; e < m; e++) {
        uint64_t x0 = mulhi64(syn_draw(seed, 2 * (uint64_t)e), tot);
        uint64_t x1 = mulhi64(syn_draw(seed, 2 * (uint64_t)e + 1), tot);
        /* upper_bound: first i with S[i] > x */
        int64_t l = 0, r = n;
        while (l < r) { int64_t md = (l + r) >> 1; if (S[md] > x0) r = md; else l = md + 1; }
        int64_t u = l;
        l = 0; r = n;
        while (l < r) { int64_t md = (l + r) >> 1; if (S[md] > x1) r = md; else l = md + 1; }
        int64_t v = l;
        if (u == v) continue;
        uint64_t a = (uint64_t)(u < v ? u : v), bb = (uint64_t)(u < v ? v : u);
        out_keys[k++] = (a << 32) | bb;
    }
    free(S);
    uint64_t *tmp = (uint64_t *)malloc(sizeof(uint64_t) * (k > 0 ? k : 1));
    radix_sort_u64(out_keys, k, tmp);
    free(tmp);
    int64_t w = 0;
    for (int64_t i = 0; i < k; i++)
        if (w == 0 || out_keys[w - 1] != out_keys[i]) out_keys[w++] = out_keys[i];
    return w;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static void sort_list(int32_t *L, int64_t len)
{
    if (len > 32) {
        qsort(L, (size_t)len, sizeof(int32_t), cmp_i32);
        return;
    }
    for (int64_t i = 1; i < len; i++) {
        int32_t x = L[i];
        int64_t j = i - 1;
        while (j >= 0 && L[j] > x) { L[j + 1] = L[j]; j--; }
        L[j + 1] = x;
    }
}

/* Symmetric CSR (each undirected edge in both lists, lists sorted) from
 * sorted unique keys (min << 32 | max).  rp: n+1, col: 2*m. */
void syn_sym_csr(int64_t n, const uint64_t *keys, int64_t m, int64_t *rp, int32_t *col)
{
    memset(rp, 0, sizeof(int64_t) * (n + 1));
    for (int64_t i = 0; i < m; i++) {
        rp[(keys[i] >> 32) + 1]++;
        rp[(keys[i] & 0xFFFFFFFFu) + 1]++;
    }
    for (int64_t v = 0; v < n; v++) rp[v + 1] += rp[v];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    memcpy(fill, rp, sizeof(int64_t) * n);
    for (int64_t i = 0; i < m; i++) {
        int64_t a = (int64_t)(keys[i] >> 32), b = (int64_t)(keys[i] & 0xFFFFFFFFu);
        col[fill[a]++] = (int32_t)b;
        col[fill[b]++] = (int32_t)a;
    }
    free(fill);
    for (int64_t v = 0; v < n; v++) {
        sort_list(col + rp[v], rp[v + 1] - rp[v]);
    }
}

/* ---- binary min-heap of 64-bit keys (degree << 32 | vertex) ---- */
typedef struct { uint64_t *a; int64_t n, cap; } heap64;

static void hpush(heap64 *h, uint64_t x)
{
    if (h->n == h->cap) {
        h->cap = h->cap ? 2 * h->cap : 1024;
        h->a = (uint64_t *)realloc(h->a, sizeof(uint64_t) * h->cap);
    }
    int64_t i = h->n++;
    while (i > 0) {
        int64_t p = (i - 1) >> 1;
        if (h->a[p] <= x) break;
        h->a[i] = h->a[p];
        i = p;
    }
    h->a[i] = x;
}

static uint64_t hpop(heap64 *h)
{
    uint64_t top = h->a[0], x = h->a[--h->n];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1;
        if (l >= h->n) break;
        int64_t r = l + 1, c = (r < h->n && h->a[r] < h->a[l]) ? r : l;
        if (h->a[c] >= x) break;
        h->a[i] = h->a[c];
        i = c;
    }
    if (h->n > 0) h->a[i] = x;
    return top;
}

/*
 * Degeneracy (smallest-last) order: repeatedly remove a vertex of minimum
 * remaining degree, the smallest id among ties.  pos[v] = removal index.
 * Returns the degeneracy (largest degree seen at removal).
 */
int64_t syn_degeneracy_order(int64_t n, const int64_t *rp, const int32_t *col, int64_t *pos)
{
    int64_t *deg = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    heap64 h = {0, 0, 0};
    for (int64_t v = 0; v < n; v++) {
        deg[v] = rp[v + 1] - rp[v];
        pos[v] = -1;
        hpush(&h, ((uint64_t)deg[v] << 32) | (uint64_t)v);
    }
    int64_t next = 0, degen = 0;
    while (h.n > 0) {
        uint64_t x = hpop(&h);
        int64_t v = (int64_t)(x & 0xFFFFFFFFu), d = (int64_t)(x >> 32);
        if (pos[v] >= 0 || d != deg[v]) continue; /* stale entry */
        pos[v] = next++;
        if (d > degen) degen = d;
        for (int64_t i = rp[v]; i < rp[v + 1]; i++) {
            int64_t u = col[i];
            if (pos[u] >= 0) continue;
            deg[u]--;
            hpush(&h, ((uint64_t)deg[u] << 32) | (uint64_t)u);
        }
    }
    free(h.a);
    free(deg);
    return degen;
}

/*
 * Orient a symmetric CSR by an order: relabel v -> pos[v], keep u -> w iff
 * pos[u] < pos[w], sort every out-list.  orp: n+1, ocol: m (undirected count).
 * Returns the largest out-degree.
 */
int64_t syn_orient(int64_t n, const int64_t *rp, const int32_t *col, const int64_t *pos,
                   int64_t *orp, int32_t *ocol)
{
    memset(orp, 0, sizeof(int64_t) * (n + 1));
    for (int64_t v = 0; v < n; v++)
        for (int64_t i = rp[v]; i < rp[v + 1]; i++)
            if (pos[v] < pos[col[i]]) orp[pos[v] + 1]++;
    int64_t maxd = 0;
    for (int64_t v = 0; v < n; v++) {
        if (orp[v + 1] > maxd) maxd = orp[v + 1];
        orp[v + 1] += orp[v];
    }
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    memcpy(fill, orp, sizeof(int64_t) * n);
    for (int64_t v = 0; v < n; v++)
        for (int64_t i = rp[v]; i < rp[v + 1]; i++)
            if (pos[v] < pos[col[i]]) ocol[fill[pos[v]]++] = (int32_t)pos[col[i]];
    free(fill);
    for (int64_t v = 0; v < n; v++) {
        sort_list(ocol + orp[v], orp[v + 1] - orp[v]);
    }
    return maxd;
}

/*
 * Induced subgraph of an oriented graph on s of its n vertices, drawn
 * uniformly without replacement with Floyd's algorithm (Bentley & Floyd,
 * CACM 1987) from the splitmix64 stream `seed`.  The chosen vertices are
 * renumbered 0..s-1 in increasing order; since the input orientation points
 * from lower to higher ids, the renumbering keeps it acyclic and every
 * out-list sorted.  Work buffers: mark (n/64 + 1 words, zero on entry and on
 * return) and map (n entries).  Output: orp[s+1], ocol[cap].  Returns the
 * number of edges, or -1 if they exceed cap.
 */
int64_t syn_induced(int64_t n, const int64_t *rp, const int32_t *col, int64_t s, uint64_t seed,
                    uint64_t *mark, int32_t *map, int64_t *orp, int32_t *ocol, int64_t cap)
{
    if (s > n) s = n;
    uint64_t e = 0;
    for (int64_t j = n - s; j < n; j++) {
        uint64_t t = mulhi64(syn_draw(seed, e++), (uint64_t)j + 1);
        if (mark[t >> 6] & (1ull << (t & 63))) t = (uint64_t)j;
        mark[t >> 6] |= 1ull << (t & 63);
    }
    int64_t k = 0;
    for (int64_t w = 0; w <= (n - 1) / 64 && n > 0; w++) {
        uint64_t b = mark[w];
        while (b) {
            int64_t v = w * 64 + __builtin_ctzll(b);
            map[v] = (int32_t)k++;
            b &= b - 1;
        }
    }
    int64_t m = 0, u_sub = 0;
    orp[0] = 0;
    for (int64_t w = 0; w <= (n - 1) / 64 && n > 0; w++) {
        uint64_t b = mark[w];
        while (b) {
            int64_t u = w * 64 + __builtin_ctzll(b);
            b &= b - 1;
            for (int64_t i = rp[u]; i < rp[u + 1]; i++) {
                int32_t v = col[i];
                if (mark[v >> 6] & (1ull << (v & 63))) {
                    if (m >= cap) {
                        memset(mark, 0, sizeof(uint64_t) * (size_t)(n / 64 + 1));
                        return -1;
                    }
                    ocol[m++] = map[v];
                }
            }
            orp[++u_sub] = m;
        }
    }
    memset(mark, 0, sizeof(uint64_t) * (size_t)(n / 64 + 1));
    return m;
}

/*
 * Plummer sphere (scale a = 1) of n points with charges, from the splitmix64
 * stream `seed`: radius by inverting the enclosed-mass fraction
 * M(r) = r^3 / (1 + r^2)^(3/2) at an open-interval uniform u, redrawn while
 * r > 100; direction uniform on the sphere (cos theta uniform in [-1, 1),
 * azimuth uniform in [0, 2 pi)); charge 2u - 1 with u open-interval uniform.
 */
static double syn_open01(uint64_t h) { return ((double)(h >> 11) + 0.5) * 0x1.0p-53; }
static double syn_unit01(uint64_t h) { return (double)(h >> 11) * 0x1.0p-53; }

void syn_plummer(int64_t n, uint64_t seed, double *x, double *y, double *z, double *q)
{
    const double two_pi = 6.283185307179586476925286766559;
    uint64_t e = 0;
    for (int64_t i = 0; i < n; i++) {
        double r;
        do {
            double u = syn_open01(syn_draw(seed, e++));
            r = 1.0 / sqrt(pow(u, -2.0 / 3.0) - 1.0);
        } while (!(r <= 100.0));
        double ct = 2.0 * syn_unit01(syn_draw(seed, e++)) - 1.0;
        double ph = two_pi * syn_unit01(syn_draw(seed, e++));
        double st = sqrt(fmax(0.0, 1.0 - ct * ct));
        x[i] = r * st * cos(ph);
        y[i] = r * st * sin(ph);
        z[i] = r * ct;
        q[i] = 2.0 * syn_open01(syn_draw(seed, e++)) - 1.0;
    }
}
