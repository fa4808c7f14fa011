/*
 * kclique_split.c -- CPU oracle of k-clique counting with cost-threshold task
 * splitting (GTaP Sec. 6.4.2, k-Clique Counting): the orientation algorithm
 * and the pivoting algorithm, with the task tree a runtime builds when a node
 * of the search becomes tasks only while its candidate set is larger than a
 * threshold.
 *
 * TEST INFRASTRUCTURE. Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  The HIP runtime never
 * calls it and shares no code with it.  Sets are plain sorted int32 vertex
 * lists here (the GPU encodes them as bitsets over the edge's candidates).
 *
 * Input: an acyclic orientation as sorted CSR out-lists N+(v).  Every
 * k-clique is counted once, at the edge (u, v) between its two lowest
 * vertices in the orientation's order: its other k-2 vertices form a
 * (k-2)-clique inside C(u, v) = N+(u) /\ N+(v).
 *
 * Task tree (k' = k - 2; t = the split threshold):
 *   R(lo,hi)  vertex range: more than `leaf` vertices -> R(lo,mid), R(mid,hi),
 *             mid = lo + (hi-lo)/2; otherwise one V(v) per vertex.
 *   V(v)      k = 1 -> 1; k = 2 -> |N+(v)|; N+(v) empty -> 0; otherwise
 *             one E(v, w) per w in N+(v) (each task explores one edge), then,
 *             resumed, the sum.
 *   E(u,v)    C = C(u,v), c = |C|.  k' = 1 -> c; c < k' -> 0; the orientation
 *             algorithm with k' = 2, or c <= t -> the root node of the chosen
 *             algorithm on C, counted in place; otherwise one child H(u,v).
 *   H(u,v)    the root node of the chosen algorithm on C as a task of its own
 *             (it holds the encoded candidate subgraph its children share).
 * Orientation (cost estimate: the candidate count):
 *   O(S, l)   counts l-cliques of the DAG induced on S (l >= 2, |S| >= l).
 *             l = 2 or |S| <= t: counted in place by
 *                 K(S,1) = |S|,  K(S,l) = sum_{x in S} K(S /\ N+(x), l-1);
 *             otherwise one child task B(S /\ N+(x), l-1) per x in S.
 *   B(S, l)   l = 1 -> |S|; |S| < l -> 0; otherwise O(S, l).
 * Pivoting (succinct clique tree of Jain and Seshadhri, WSDM 2020; the graph
 * inside C is undirected: x ~ y when either is in the other's out-list; the
 * cost estimate is the size of the candidate set):
 *   P(Q, h, q) counts the cliques of size k' made of the h "held" vertices of
 *             the path to this node, any q' of its q pivots and a clique of
 *             the candidates Q:
 *             h = k' -> 1; Q empty -> binom(q, k'-h); q + |Q| < k'-h -> 0;
 *             |Q| <= t: counted in place by the same recursion;
 *             otherwise the pivot p is the candidate with the most neighbours
 *             in Q (the lowest position on ties), and the children are
 *               P(Q /\ N(p), h, q+1)                          (p as pivot)
 *               P(Q_i /\ N(w_i), h+1, q) for the members w_1 < w_2 < ... of
 *               Q \ N(p) other than p, Q_i = Q minus p, w_1, ..., w_{i-1}.
 *             Done in place, the children are recursive calls instead.
 *             (Adjacency inside C is tabulated once per edge.)
 * Every child listed is one task; a task with children suspends once
 * (conts).  aux counts the nodes that split (O or P nodes with children,
 * the edge's root node included).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t tasks, conts, leaves, aux;
} ks_counts;

typedef struct {
    const int64_t *rp;
    const int32_t *col;
    int k;          /* clique size */
    int kk;         /* k - 2 */
    int thr;        /* split threshold */
    int pivot;      /* 0: orientation, 1: pivoting */
    int bad;        /* allocation failure */
    ks_counts *c;
    const char *adj;  /* pivoting: c x c adjacency of the current edge's candidates */
    int64_t nadj;
} ks_ctx;

static int64_t ks_isect(const int32_t *a, int64_t na, const int32_t *b, int64_t nb, int32_t *out)
{
    int64_t i = 0, j = 0, o = 0;
    while (i < na && j < nb) {
        if (a[i] < b[j]) i++;
        else if (a[i] > b[j]) j++;
        else {
            if (out) out[o] = a[i];
            o++;
            i++;
            j++;
        }
    }
    return o;
}

static int ks_has(const int32_t *a, int64_t na, int32_t x)
{
    int64_t lo = 0, hi = na;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo < na && a[lo] == x;
}

static const int32_t *ks_out(const ks_ctx *x, int32_t v, int64_t *len)
{
    *len = x->rp[v + 1] - x->rp[v];
    return x->col + x->rp[v];
}

/* x ~ y inside a candidate set: an edge in either direction */
static int ks_adj(const ks_ctx *x, int32_t a, int32_t b)
{
    int64_t na, nb;
    const int32_t *oa = ks_out(x, a, &na), *ob = ks_out(x, b, &nb);
    return ks_has(oa, na, b) || ks_has(ob, nb, a);
}

/* C(n, r) exactly (the count must fit int64) */
static int64_t ks_binom(int64_t n, int64_t r)
{
    if (r < 0 || r > n) return 0;
    unsigned __int128 v = 1;
    for (int64_t i = 1; i <= r; i++) v = v * (unsigned __int128)(n - r + i) / (unsigned __int128)i;
    return (int64_t)v;
}

static void *ks_alloc(ks_ctx *x, size_t n)
{
    void *p = calloc(n > 0 ? n : 1, 1);
    if (!p) x->bad = 1;
    return p;
}

/* ---- orientation ---------------------------------------------------------- */

/* K(S, l) by plain recursion */
static int64_t ks_K(ks_ctx *x, const int32_t *S, int64_t ns, int l)
{
    if (l == 1) return ns;
    int32_t *T = ks_alloc(x, sizeof(int32_t) * (size_t)ns);
    if (!T) return 0;
    int64_t sum = 0;
    for (int64_t i = 0; i < ns; i++) {
        int64_t nu;
        const int32_t *ou = ks_out(x, S[i], &nu);
        int64_t nt = ks_isect(S, ns, ou, nu, T);
        if (nt >= l - 1) sum += ks_K(x, T, nt, l - 1);
    }
    free(T);
    return sum;
}

static int64_t ks_B(ks_ctx *x, const int32_t *S, int64_t ns, int l);

static int64_t ks_O(ks_ctx *x, const int32_t *S, int64_t ns, int l)
{
    if (l == 2 || ns <= x->thr) return ks_K(x, S, ns, l);
    x->c->aux++;
    int32_t *T = ks_alloc(x, sizeof(int32_t) * (size_t)ns);
    if (!T) return 0;
    int64_t sum = 0;
    for (int64_t i = 0; i < ns; i++) {
        int64_t nu;
        const int32_t *ou = ks_out(x, S[i], &nu);
        int64_t nt = ks_isect(S, ns, ou, nu, T);
        sum += ks_B(x, T, nt, l - 1);
    }
    free(T);
    x->c->conts++;
    return sum;
}

static int64_t ks_B(ks_ctx *x, const int32_t *S, int64_t ns, int l)
{
    x->c->tasks++;
    if (l == 1) {
        x->c->leaves++;
        return ns;
    }
    if (ns < l) {
        x->c->leaves++;
        return 0;
    }
    int64_t before = x->c->conts;
    int64_t v = ks_O(x, S, ns, l);
    if (x->c->conts == before) x->c->leaves++;
    return v;
}

/* ---- pivoting ------------------------------------------------------------- */

/* One node of the clique tree.  Q holds positions in the edge's candidate
 * list (ascending), adjacency comes from x->adj.  `task` = 1 when the node is
 * a task of its own (then its children may be tasks too); in place otherwise. */
static int ks_nb(const ks_ctx *x, int32_t a, int32_t b) { return x->adj[(int64_t)a * x->nadj + b]; }

static int64_t ks_P(ks_ctx *x, const int32_t *Q, int64_t nq, int h, int q, int task)
{
    const int kk = x->kk;
    if (h == kk) return 1;
    if (nq == 0) return ks_binom(q, kk - h);
    if (q + nq < kk - h) return 0;
    const int split = task && nq > x->thr;
    /* pivot: most neighbours inside Q, lowest position on ties */
    int64_t best = -1, pbest = 0;
    for (int64_t i = 0; i < nq; i++) {
        int64_t d = 0;
        for (int64_t j = 0; j < nq; j++)
            if (j != i && ks_nb(x, Q[i], Q[j])) d++;
        if (d > best) {
            best = d;
            pbest = i;
        }
    }
    const int32_t p = Q[pbest];
    int32_t *T = ks_alloc(x, sizeof(int32_t) * (size_t)nq);
    char *gone = ks_alloc(x, (size_t)nq);
    if (!T || !gone) {
        free(T);
        free(gone);
        return 0;
    }
    if (split) x->c->aux++;
    int64_t sum = 0;
    /* p as pivot */
    int64_t nt = 0;
    for (int64_t j = 0; j < nq; j++)
        if (j != pbest && ks_nb(x, p, Q[j])) T[nt++] = Q[j];
    if (split) x->c->tasks++;
    int64_t before = x->c->conts;
    sum += ks_P(x, T, nt, h, q + 1, split);
    if (split && x->c->conts == before) x->c->leaves++;
    gone[pbest] = 1;
    /* the non-neighbours of p, each held, in ascending order */
    for (int64_t i = 0; i < nq; i++) {
        if (i == pbest || ks_nb(x, p, Q[i])) continue;
        nt = 0;
        for (int64_t j = 0; j < nq; j++)
            if (!gone[j] && j != i && ks_nb(x, Q[i], Q[j])) T[nt++] = Q[j];
        if (split) x->c->tasks++;
        before = x->c->conts;
        sum += ks_P(x, T, nt, h + 1, q, split);
        if (split && x->c->conts == before) x->c->leaves++;
        gone[i] = 1;
    }
    free(T);
    free(gone);
    if (split) x->c->conts++;
    return sum;
}

/* ---- task tree above the algorithms --------------------------------------- */

/* root node of an edge's search; task = 1 when it is a task of its own.
 * Pivoting works on candidate positions 0..c-1 with the undirected adjacency
 * of the candidates tabulated first. */
static int64_t ks_root(ks_ctx *x, const int32_t *C, int64_t c, int task)
{
    if (!x->pivot) return task ? ks_O(x, C, c, x->kk) : ks_K(x, C, c, x->kk);
    char *adj = ks_alloc(x, (size_t)(c * c));
    int32_t *Q = ks_alloc(x, sizeof(int32_t) * (size_t)c);
    int64_t r = 0;
    if (adj && Q) {
        for (int64_t i = 0; i < c; i++) {
            Q[i] = (int32_t)i;
            for (int64_t j = 0; j < c; j++) adj[i * c + j] = (char)(i != j && ks_adj(x, C[i], C[j]));
        }
        x->adj = adj;
        x->nadj = c;
        r = ks_P(x, Q, c, 0, 0, task);
    }
    free(adj);
    free(Q);
    return r;
}

static int64_t ks_E(ks_ctx *x, int32_t u, int32_t v)
{
    x->c->tasks++;
    int64_t nu, nv;
    const int32_t *ou = ks_out(x, u, &nu), *ov = ks_out(x, v, &nv);
    int32_t *C = ks_alloc(x, sizeof(int32_t) * (size_t)(nu < nv ? nu : nv));
    if (!C) return 0;
    int64_t c = ks_isect(ou, nu, ov, nv, C);
    int64_t r;
    if (x->kk == 1) r = c;
    else if (c < x->kk) r = 0;
    else if (c <= x->thr || (!x->pivot && x->kk == 2)) r = ks_root(x, C, c, 0);
    else {
        /* H(u, v) */
        x->c->tasks++;
        int64_t before = x->c->conts;
        r = ks_root(x, C, c, 1);
        if (x->c->conts == before) x->c->leaves++;
        x->c->conts++;
        free(C);
        return r;
    }
    x->c->leaves++;
    free(C);
    return r;
}

static int64_t ks_V(ks_ctx *x, int32_t v)
{
    x->c->tasks++;
    int64_t nv;
    const int32_t *ov = ks_out(x, v, &nv);
    if (x->k == 1) {
        x->c->leaves++;
        return 1;
    }
    if (x->k == 2 || nv == 0) {
        x->c->leaves++;
        return x->k == 2 ? nv : 0;
    }
    int64_t sum = 0;
    for (int64_t i = 0; i < nv; i++) sum += ks_E(x, v, ov[i]);
    x->c->conts++;
    return sum;
}

static int64_t ks_R(ks_ctx *x, int64_t lo, int64_t hi, int64_t leaf)
{
    x->c->tasks++;
    if (hi - lo <= 0) {
        x->c->leaves++;
        return 0;
    }
    int64_t sum = 0;
    if (hi - lo > leaf) {
        int64_t mid = lo + (hi - lo) / 2;
        sum += ks_R(x, lo, mid, leaf);
        sum += ks_R(x, mid, hi, leaf);
    } else {
        for (int64_t v = lo; v < hi; v++) sum += ks_V(x, (int32_t)v);
    }
    x->c->conts++;
    return sum;
}

/* Returns the number of k-cliques, -1 on invalid arguments, -2 when out of
 * memory.  algorithm: 0 orientation, 1 pivoting.  threshold >= 0. */
int64_t orc_kclique_split(const int64_t *row_ptr, const int32_t *col, int64_t n, int k,
                          int64_t range_leaf, int threshold, int algorithm, ks_counts *c)
{
    memset(c, 0, sizeof(*c));
    if (k < 1 || n < 0 || range_leaf < 1 || threshold < 0 || (algorithm != 0 && algorithm != 1)) return -1;
    ks_ctx x = {row_ptr, col, k, k - 2, threshold, algorithm, 0, c, NULL, 0};
    int64_t v = ks_R(&x, 0, n, range_leaf);
    return x.bad ? -2 : v;
}

/* The same count restricted to the cliques whose lowest vertex v satisfies
 * v % stride == offset (a sample of vertex tasks for timing; summing over
 * every offset gives the full count).  Task counts cover those vertex
 * subtrees only. */
int64_t orc_kclique_split_roots(const int64_t *row_ptr, const int32_t *col, int64_t n, int k,
                                int64_t stride, int64_t offset, int threshold, int algorithm,
                                ks_counts *c)
{
    memset(c, 0, sizeof(*c));
    if (k < 1 || n < 0 || stride < 1 || offset < 0 || offset >= stride || threshold < 0 ||
        (algorithm != 0 && algorithm != 1))
        return -1;
    ks_ctx x = {row_ptr, col, k, k - 2, threshold, algorithm, 0, c, NULL, 0};
    int64_t sum = 0;
    for (int64_t v = offset; v < n; v += stride) sum += ks_V(&x, (int32_t)v);
    return x.bad ? -2 : sum;
}
