/*
 * oracle.c -- plain, sequential CPU oracle for the GTaP fork-join workloads.
 *
 * TEST INFRASTRUCTURE. Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  The HIP runtime never
 * calls it and shares no code, header, table or constant generator with it.
 *
 * Every function below is the textbook recursive definition of a workload, run
 * depth-first on one core.  Besides the result it counts what the fork-join
 * formulation executes (GTaP Sec. 5.1.2, "Implementation of Fork-Join"):
 *   tasks  -- one per task call (every recursive call is a task, no cutoff);
 *   conts  -- one per resumption: a task that forked at least one child
 *             suspends at its join and is executed once more after the last
 *             child completes (the join is implicit at task return).
 * The fork tree does not depend on the schedule, so tasks + conts is an exact
 * target for the number of executions any correct runtime performs.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>

typedef struct {
    int64_t tasks;   /* task calls */
    int64_t conts;   /* resumptions after a join */
    int64_t leaves;  /* workload-specific: tasks with no children */
    int64_t aux;     /* workload-specific (UTS: deepest level reached) */
} orc_counts;

/* ---------------------------------------------------------------------------
 * Fibonacci, one task per call, no cutoff (Sec. 6.3, Fibonacci microbenchmark:
 * in the comparison every recursive call is a task of its own).
 * fib(n) = n for n < 2, else fib(n-1) + fib(n-2).
 * ------------------------------------------------------------------------- */
static int64_t fib_rec(int n, orc_counts *c)
{
    c->tasks++;
    if (n < 2) {
        c->leaves++;
        return n;
    }
    int64_t a = fib_rec(n - 1, c);
    int64_t b = fib_rec(n - 2, c);
    c->conts++;
    return a + b;
}

int64_t orc_fib(int n, orc_counts *c)
{
    memset(c, 0, sizeof(*c));
    if (n < 0) return -1;
    return fib_rec(n, c);
}

/* ---------------------------------------------------------------------------
 * N-Queens by bitmask backtracking (Sec. 6.3, N-Queens microbenchmark: counts
 * solutions via bitmask-based backtracking).  A node is the set of queens on
 * rows [0,row); its children place one queen on each column of row `row` not
 * attacked along a column or a diagonal.  A full board counts 1, a dead end 0.
 * Every node is a task (no cutoff).
 * ------------------------------------------------------------------------- */
static int64_t nq_rec(uint32_t full, uint32_t cols, uint32_t dl, uint32_t dr,
                      int row, int n, orc_counts *c)
{
    c->tasks++;
    if (row == n) {
        c->leaves++;
        return 1;
    }
    uint32_t avail = full & ~(cols | dl | dr);
    if (avail == 0) {
        c->leaves++;
        return 0;
    }
    int64_t sum = 0;
    for (int col = 0; col < n; col++) {
        uint32_t b = 1u << col;
        if (!(avail & b)) continue;
        sum += nq_rec(full, cols | b, ((dl | b) << 1) & full, (dr | b) >> 1,
                      row + 1, n, c);
    }
    c->conts++;
    return sum;
}

int64_t orc_nqueens(int n, orc_counts *c)
{
    memset(c, 0, sizeof(*c));
    if (n < 1 || n > 30) return -1;
    uint32_t full = (n == 32) ? 0xFFFFFFFFu : ((1u << n) - 1u);
    return nq_rec(full, 0, 0, 0, 0, n, c);
}

/* ---------------------------------------------------------------------------
 * Unbalanced tree search.  The paper names no UTS definition; this is the
 * binomial-free geometric variant: a node (id, depth) has no children at the
 * depth limit, otherwise its child count is the number of leading draws
 * j = 1, 2, ... whose hash falls below an integer threshold T, i.e. a geometric
 * law on {0,1,...} with continue-probability T / 2^64 (mean m when
 * T = floor(2^64 m / (m+1))).  Child i of node id has id split(id, i).
 *
 * The hash is splitmix64's output function, written here from its published
 * definition (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014): add the golden gamma, then two xor-shift-multiply
 * rounds and a final xor-shift.
 * ------------------------------------------------------------------------- */
#define ORC_GOLDEN_GAMMA 0x9E3779B97F4A7C15ull
#define ORC_UTS_DRAW_KEY 0xD1B54A32D192ED03ull

static uint64_t orc_mix64(uint64_t z)
{
    z += ORC_GOLDEN_GAMMA;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint64_t orc_split(uint64_t a, uint64_t i)
{
    return orc_mix64(a + (i + 1) * ORC_GOLDEN_GAMMA);
}

uint64_t orc_uts_mix64(uint64_t z) { return orc_mix64(z); }

int orc_uts_num_children(uint64_t id, int depth, uint64_t thr, int max_depth)
{
    if (depth >= max_depth) return 0;
    int c = 0;
    for (uint64_t j = 1;; j++) {
        if (orc_mix64(id ^ (j * ORC_UTS_DRAW_KEY)) < thr) c++;
        else break;
    }
    return c;
}

static int64_t uts_rec(uint64_t id, int depth, uint64_t thr, int max_depth,
                       orc_counts *c)
{
    c->tasks++;
    if (depth > c->aux) c->aux = depth;
    int nc = orc_uts_num_children(id, depth, thr, max_depth);
    if (nc == 0) {
        c->leaves++;
        return 1;
    }
    int64_t sum = 1;
    for (int i = 0; i < nc; i++)
        sum += uts_rec(orc_split(id, (uint64_t)i), depth + 1, thr, max_depth, c);
    c->conts++;
    return sum;
}

/* Returns the number of nodes of the tree rooted at id = mix64(seed). */
int64_t orc_uts(uint64_t seed, uint64_t thr, int max_depth, orc_counts *c)
{
    memset(c, 0, sizeof(*c));
    if (max_depth < 0) return -1;
    return uts_rec(orc_mix64(seed), 0, thr, max_depth, c);
}

/* ---------------------------------------------------------------------------
 * k-clique counting by graph orientation (Sec. 6.4.2, k-Clique Counting,
 * orientation algorithm).  On a DAG whose out-lists N+(v) are sorted, every
 * k-clique is counted once from its lowest vertex:
 *     K(C, 1) = |C|,   K(C, l) = sum_{u in C} K(C /\ N+(u), l-1),
 *     total   = sum_v K(N+(v), k-1)            (k >= 2; k = 1 gives n).
 *
 * Task tree (one task per recursive call, counted so the GPU runtime can be
 * checked execution by execution):
 *   R(lo,hi)  vertex-range root: more than `leaf` vertices -> two children
 *             R(lo,mid), R(mid,hi) with mid = lo + (hi-lo)/2; otherwise one
 *             child V(v) per vertex of the range.
 *   V(v)      k = 1 -> 1; k = 2 -> |N+(v)|; else one child T(N+(v), u, k-2)
 *             per u in N+(v).
 *   T(C,u,l)  C' = C /\ N+(u); l = 1 -> |C'|; else one child T(C', w, l-1)
 *             per w in C'.
 * ------------------------------------------------------------------------- */
static int64_t isect_sorted(const int32_t *a, int64_t na, const int32_t *b,
                            int64_t nb, int32_t *out)
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

typedef struct {
    const int64_t *row_ptr;
    const int32_t *col;
    int k;
    int32_t *scratch;  /* (k) * max_outdeg int32 */
    int64_t stride;
    orc_counts *c;
} kc_ctx;

static int64_t kc_T(kc_ctx *x, const int32_t *C, int64_t nC, int32_t u, int l,
                    int depth)
{
    x->c->tasks++;
    const int32_t *nu = x->col + x->row_ptr[u];
    int64_t nnu = x->row_ptr[u + 1] - x->row_ptr[u];
    if (l == 1) {
        x->c->leaves++;
        return isect_sorted(C, nC, nu, nnu, NULL);
    }
    int32_t *Cp = x->scratch + (int64_t)depth * x->stride;
    int64_t nCp = isect_sorted(C, nC, nu, nnu, Cp);
    if (nCp == 0) {
        x->c->leaves++;
        return 0;
    }
    int64_t sum = 0;
    for (int64_t i = 0; i < nCp; i++)
        sum += kc_T(x, Cp, nCp, Cp[i], l - 1, depth + 1);
    x->c->conts++;
    return sum;
}

static int64_t kc_V(kc_ctx *x, int32_t v)
{
    x->c->tasks++;
    const int32_t *C = x->col + x->row_ptr[v];
    int64_t nC = x->row_ptr[v + 1] - x->row_ptr[v];
    if (x->k == 1) {
        x->c->leaves++;
        return 1;
    }
    if (x->k == 2) {
        x->c->leaves++;
        return nC;
    }
    if (nC == 0) {
        x->c->leaves++;
        return 0;
    }
    int64_t sum = 0;
    for (int64_t i = 0; i < nC; i++) sum += kc_T(x, C, nC, C[i], x->k - 2, 0);
    x->c->conts++;
    return sum;
}

static int64_t kc_R(kc_ctx *x, int64_t lo, int64_t hi, int64_t leaf)
{
    x->c->tasks++;
    if (hi - lo <= 0) {
        x->c->leaves++;
        return 0;
    }
    int64_t sum = 0;
    if (hi - lo > leaf) {
        int64_t mid = lo + (hi - lo) / 2;
        sum += kc_R(x, lo, mid, leaf);
        sum += kc_R(x, mid, hi, leaf);
    } else {
        for (int64_t v = lo; v < hi; v++) sum += kc_V(x, (int32_t)v);
    }
    x->c->conts++;
    return sum;
}

/* row_ptr has n+1 entries; out-lists must be sorted ascending and acyclic
 * (u -> w implies u precedes w in some order).  scratch must hold
 * max(k-2,1) * max_outdeg int32.  Returns the number of k-cliques, or -1. */
int64_t orc_kclique(const int64_t *row_ptr, const int32_t *col, int64_t n,
                    int k, int64_t range_leaf, int32_t *scratch,
                    int64_t max_outdeg, orc_counts *c)
{
    memset(c, 0, sizeof(*c));
    if (k < 1 || n < 0 || range_leaf < 1) return -1;
    kc_ctx x = {row_ptr, col, k, scratch, max_outdeg > 0 ? max_outdeg : 1, c};
    return kc_R(&x, 0, n, range_leaf);
}
