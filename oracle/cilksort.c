/*
 * cilksort.c -- plain, sequential CPU oracle of the Cilksort microbenchmark
 * (GTaP Sec. 6.3, "Workloads": a mergesort whose merges are themselves split
 * in parallel, with a sort cutoff and a merge cutoff).
 *
 * TEST INFRASTRUCTURE. Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  The HIP runtime never
 * calls it and shares no code with it.
 *
 * Reading of the recursion (the paper names the benchmark and its two
 * cutoffs only):
 *   sort(lo, n, dst): the keys x[lo, lo+n) end up sorted in buffer dst (x or
 *     the scratch buffer t).  n <= sort_cutoff: a serial sort of a copy;
 *     otherwise sort the halves [lo, lo+n/2) and the rest into the other
 *     buffer, then merge them from there into dst.
 *   merge(S, A, B, D, d0): the sorted ranges A and B of buffer S merged into
 *     D[d0, ...).  The longer range is A (swap if B is longer).  If
 *     |A| + |B| <= merge_cutoff: a serial two-way merge; otherwise A's middle
 *     element v = A[|A|/2] splits A, the number of elements of B below v
 *     splits B, and the two lower parts and the two upper parts are merged
 *     independently (the upper parts start at d0 + |A_low| + |B_low|).
 * Every call is a task; an internal sort resumes twice (after its two sorts,
 * after its merge), an internal merge once (after its two merges).  The fork
 * tree depends on the keys but not on the schedule.
 */
#include <stdint.h>
#include <string.h>

typedef struct {
    int64_t tasks;
    int64_t conts;
    int64_t leaves;
    int64_t aux;   /* merge tasks */
} orc_counts;

typedef struct {
    uint32_t *x, *t;
    int64_t sort_cut, merge_cut;
    orc_counts *c;
} cs_ctx;

static void cs_merge(cs_ctx *k, const uint32_t *S, int64_t a0, int64_t na, int64_t b0, int64_t nb,
                     uint32_t *D, int64_t d0)
{
    k->c->tasks++;
    k->c->aux++;
    if (nb > na) {
        int64_t s = a0; a0 = b0; b0 = s;
        s = na; na = nb; nb = s;
    }
    if (na + nb <= k->merge_cut) {
        int64_t i = 0, j = 0, o = d0;
        while (i < na && j < nb) D[o++] = (S[b0 + j] < S[a0 + i]) ? S[b0 + j++] : S[a0 + i++];
        while (i < na) D[o++] = S[a0 + i++];
        while (j < nb) D[o++] = S[b0 + j++];
        k->c->leaves++;
        return;
    }
    const int64_t ma = na / 2;
    const uint32_t v = S[a0 + ma];
    int64_t mb = 0;
    while (mb < nb && S[b0 + mb] < v) ++mb;   /* plain linear count of B's keys below v */
    cs_merge(k, S, a0, ma, b0, mb, D, d0);
    cs_merge(k, S, a0 + ma, na - ma, b0 + mb, nb - mb, D, d0 + ma + mb);
    k->c->conts++;
}

static void cs_sort(cs_ctx *k, int64_t lo, int64_t n, int dst)
{
    k->c->tasks++;
    uint32_t *D = dst ? k->t : k->x;
    if (n <= k->sort_cut) {
        /* serial sort: insertion sort of a copy */
        for (int64_t i = 0; i < n; ++i) {
            const uint32_t v = k->x[lo + i];
            int64_t j = i;
            while (j > 0 && D[lo + j - 1] > v) {
                D[lo + j] = D[lo + j - 1];
                --j;
            }
            D[lo + j] = v;
        }
        k->c->leaves++;
        return;
    }
    const int64_t h = n / 2;
    cs_sort(k, lo, h, !dst);
    cs_sort(k, lo + h, n - h, !dst);
    k->c->conts++;
    cs_merge(k, dst ? k->x : k->t, lo, h, lo + h, n - h, D, lo);
    k->c->conts++;
}

/* Sort x[0, n) in place (t: scratch of n keys).  Returns n. */
int64_t orc_cilksort(uint32_t *x, uint32_t *t, int64_t n, int64_t sort_cut, int64_t merge_cut, orc_counts *c)
{
    cs_ctx k = {x, t, sort_cut, merge_cut, c};
    memset(c, 0, sizeof(*c));
    cs_sort(&k, 0, n, 0);
    return n;
}
