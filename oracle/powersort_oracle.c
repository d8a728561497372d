/*
 * Powersort oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU implementation of powersort as defined in
 * Munro & Wild, "Nearly-Optimal Mergesorts: Fast, Practical Sorting Methods
 * That Optimally Adapt to Existing Runs" (ESA 2018, arXiv:1805.04154).  Only
 * the test suite, the package smoke check and the CPU-baseline leg of the
 * benchmark may load this library; the product path never does, and this file
 * shares no code, header or table with the GPU implementation.
 *
 * It follows the paper's steps in the paper's order (Alg. PowerSort in
 * Sec. 3.2.2, with the minimum-run-length extension of App. B.4):
 *   1. find the next run by a left-to-right scan under the run convention of
 *      Sec. 2: a maximal weakly increasing block, or a strictly decreasing
 *      block that is reversed at once;
 *   2. if that run is shorter than the minimum run length w, extend it to
 *      min(n, start + w) elements by straight insertion sort with a presorted
 *      prefix (App. B.3);
 *   3. compute the power of the boundary between the previous run and this one
 *      by the defining loop of Def. "Node Power" / procedure NodePower, in
 *      exact integer arithmetic (the paper's real-valued midpoints, scaled by
 *      2n, are integers);
 *   4. while the power on top of the stack exceeds the new power, pop and
 *      merge the popped run with the current run; then push;
 *   5. at the end merge everything left on the stack;
 * merging stably, taking from the right run only when its head is strictly
 * smaller (App. B.1), and charging each merge its result size (Sec. 2.2).
 *
 * The file also holds peeksort (Alg. PeekSort, Sec. 3.1) over the same leaves;
 * see the section at the end.
 *
 * Parity status: pinned (see the tests' oracle-pin suite): the output against
 * a library stable sort, the run partition against two other formulations of
 * the run convention, the powers against the paper's Fig. 1 values and an
 * exact-rational evaluation, the merge list against the Cartesian tree of the
 * powers (Cor. "Cartesian tree"), and the merge cost against Fig. 1, the
 * entropy bounds of Thm. "powersort" and an interval-DP optimum.  The
 * galloping merge is pinned by equality with the plain merge's result and
 * merge cost, the information bound on comparisons per merge, equality with
 * the plain count on alternating merges, and a logarithmic cost per block on
 * block merges.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Key types.  The numbering is this file's own. */
enum { ORK_I32 = 0, ORK_U32 = 1, ORK_I64 = 2, ORK_U64 = 3, ORK_F32 = 4 };

typedef struct {
    unsigned char *key; /* n keys of ks bytes each */
    uint32_t *pay;      /* n payload words, or NULL */
    size_t ks;          /* key size in bytes */
    int type;
} arr_t;

typedef struct {
    uint64_t lo, mid, hi; /* a merge of [lo, mid) and [mid, hi) */
} ora_merge;

/* IEEE-754 totalOrder on binary32 bit patterns: -NaN < -inf < ... < -0 <
 * +0 < ... < +inf < +NaN, NaNs ordered by their payload. */
static int f32_total_less(uint32_t a, uint32_t b) {
    int sa = (int)(a >> 31), sb = (int)(b >> 31);
    if (sa != sb) return sa > sb; /* the negative one is smaller */
    if (!sa) return a < b;        /* both non-negative: larger bits, larger value */
    return a > b;                 /* both negative: larger magnitude, smaller value */
}

/* Key comparisons made by the calling thread's last oracle_powersort /
 * oracle_peeksort call (Thm. "powersort" / "peeksort" bound them); every
 * comparison goes through key_less.  Each call runs on one thread; the count
 * is per thread so that independent calls may run on several threads. */
static _Thread_local uint64_t g_comparisons;

/* key_less(x, y): the key stored at x orders strictly before the key at y. */
static int key_less(const arr_t *A, const unsigned char *x, const unsigned char *y) {
    g_comparisons++;
    switch (A->type) {
    case ORK_I32: { int32_t a, b; memcpy(&a, x, 4); memcpy(&b, y, 4); return a < b; }
    case ORK_U32: { uint32_t a, b; memcpy(&a, x, 4); memcpy(&b, y, 4); return a < b; }
    case ORK_I64: { int64_t a, b; memcpy(&a, x, 8); memcpy(&b, y, 8); return a < b; }
    case ORK_U64: { uint64_t a, b; memcpy(&a, x, 8); memcpy(&b, y, 8); return a < b; }
    case ORK_F32: { uint32_t a, b; memcpy(&a, x, 4); memcpy(&b, y, 4); return f32_total_less(a, b); }
    }
    return 0;
}

static int less_at(const arr_t *A, uint64_t i, uint64_t j) {
    return key_less(A, A->key + i * A->ks, A->key + j * A->ks);
}

static void swap_at(arr_t *A, uint64_t i, uint64_t j) {
    unsigned char t[8];
    memcpy(t, A->key + i * A->ks, A->ks);
    memcpy(A->key + i * A->ks, A->key + j * A->ks, A->ks);
    memcpy(A->key + j * A->ks, t, A->ks);
    if (A->pay) { uint32_t p = A->pay[i]; A->pay[i] = A->pay[j]; A->pay[j] = p; }
}

/* Reverse A[s..e). */
static void reverse_range(arr_t *A, uint64_t s, uint64_t e) {
    while (e > s + 1) { swap_at(A, s, e - 1); s++; e--; }
}

/* ExtendRunRight (Sec. 2 run convention, Alg. PowerSort): return e such that
 * A[s..e) is the run that starts at s.  A run is weakly increasing, or
 * strictly decreasing; a strictly decreasing run is reversed in place, which
 * is stable because it holds no equal keys. */
static uint64_t extend_run_right(arr_t *A, uint64_t s, uint64_t n) {
    uint64_t e = s + 1;
    if (e < n && less_at(A, e, e - 1)) {
        e++;  /* each adjacent pair is compared once */
        while (e < n && less_at(A, e, e - 1)) e++;
        reverse_range(A, s, e);
    } else if (e < n) {
        e++;
        while (e < n && !less_at(A, e, e - 1)) e++;
    }
    return e;
}

/* Straight insertion sort of A[s..e) whose first k elements are already
 * sorted (App. B.3).  An element moves left only past strictly larger keys,
 * which keeps the sort stable. */
static void insertion_sort(arr_t *A, uint64_t s, uint64_t e, uint64_t k) {
    unsigned char v[8];
    for (uint64_t i = s + k; i < e; i++) {
        memcpy(v, A->key + i * A->ks, A->ks);
        uint32_t pv = A->pay ? A->pay[i] : 0;
        uint64_t j = i;
        while (j > s && key_less(A, v, A->key + (j - 1) * A->ks)) {
            memcpy(A->key + j * A->ks, A->key + (j - 1) * A->ks, A->ks);
            if (A->pay) A->pay[j] = A->pay[j - 1];
            j--;
        }
        memcpy(A->key + j * A->ks, v, A->ks);
        if (A->pay) A->pay[j] = pv;
    }
}

/* Def. "Node Power" / procedure NodePower: the smallest l with
 * floor(a 2^l) != floor(b 2^l), where a and b are the midpoints of the two
 * runs divided by n.  With 0-based starts s1, s2 and lengths n1, n2 the
 * midpoints scaled by 2n are the integers 2 s1 + n1 and 2 s2 + n2, so
 * floor(a 2^l) = floor((2 s1 + n1) 2^l / (2n)) exactly. */
static unsigned node_power(uint64_t s1, uint64_t n1, uint64_t s2, uint64_t n2, uint64_t n) {
    unsigned __int128 an = 2 * (unsigned __int128)s1 + n1;
    unsigned __int128 bn = 2 * (unsigned __int128)s2 + n2;
    unsigned __int128 d = 2 * (unsigned __int128)n;
    unsigned l = 0;
    while ((an << l) / d == (bn << l) / d) l++;
    return l;
}

/* Merge(A[lo..mid), A[mid..hi)) stably through buffer tmp (App. B.1): the
 * right run's head is taken only when it is strictly smaller. */
static void merge_runs(arr_t *A, uint64_t lo, uint64_t mid, uint64_t hi,
                       unsigned char *tk, uint32_t *tp) {
    uint64_t i = lo, j = mid, o = 0;
    size_t ks = A->ks;
    while (i < mid || j < hi) {
        int take_right = (i >= mid) || (j < hi && less_at(A, j, i));
        uint64_t src = take_right ? j++ : i++;
        memcpy(tk + o * ks, A->key + src * ks, ks);
        if (A->pay) tp[o] = A->pay[src];
        o++;
    }
    memcpy(A->key + lo * ks, tk, (hi - lo) * ks);
    if (A->pay) memcpy(A->pay + lo, tp, (hi - lo) * sizeof(uint32_t));
}

/* Galloping merge (the comparison-saving merge of Timsort that Sec. 4.1
 * describes and Sec. 5 names for future comparison-efficient merging): a
 * plain merge that counts how many times in a row each run has supplied the
 * output; once one run has won kGallop times in a row it switches to
 * exponential searches -- the number of left elements not above the right
 * head, then the number of right elements below the left head -- and copies
 * those blocks whole, until both searches return fewer than kGallop
 * elements.  Equal keys still go left first, so the result is exactly
 * merge_runs's; only the comparisons differ.  The paper fixes no threshold;
 * kGallop = 7 is Timsort's.  (Peters' adaptive threshold is not used.) */
enum { kGallop = 7 };

/* Exponential then binary search: the number of elements of A[s..e) that
 * precede key v in a stable merge where A is the LEFT run (those not above
 * v: !(v < x)) if left_run, else where A is the RIGHT run (those strictly
 * below v). */
static uint64_t gallop_count(const arr_t *A, uint64_t s, uint64_t e, const unsigned char *v, int left_run) {
    uint64_t lo = 0, hi = 1, len = e - s;  /* the count lies in (lo - 1 ... ] as probed */
    /* goes(k): element s + k precedes v */
    #define GOES(k) (left_run ? !key_less(A, v, A->key + (s + (k)) * A->ks) \
                              : key_less(A, A->key + (s + (k)) * A->ks, v))
    if (len == 0 || !GOES(0)) return 0;
    /* invariant: elements [0, lo] go; probe lo + hi */
    while (lo + hi < len && GOES(lo + hi)) { lo += hi; hi *= 2; }
    /* elements [0, lo] go; element min(lo + hi, len) does not (or is past the end) */
    uint64_t a = lo + 1, b = (lo + hi < len) ? lo + hi : len;  /* count in [a, b] */
    while (a < b) {
        uint64_t m = a + (b - a) / 2;  /* does element m go? */
        if (GOES(m)) a = m + 1; else b = m;
    }
    #undef GOES
    return a;
}

/* Append element src to the merge buffer at o. */
static void take_one(const arr_t *A, uint64_t src, unsigned char *tk, uint32_t *tp, uint64_t *o) {
    memcpy(tk + *o * A->ks, A->key + src * A->ks, A->ks);
    if (A->pay) tp[*o] = A->pay[src];
    (*o)++;
}

static void merge_runs_galloping(arr_t *A, uint64_t lo, uint64_t mid, uint64_t hi,
                                 unsigned char *tk, uint32_t *tp) {
    uint64_t i = lo, j = mid, o = 0;
    size_t ks = A->ks;
    unsigned wins_left = 0, wins_right = 0;
#define TAKE(src) take_one(A, (src), tk, tp, &o)
    while (i < mid && j < hi) {
        if (wins_left < kGallop && wins_right < kGallop) {
            if (less_at(A, j, i)) { TAKE(j); j++; wins_right++; wins_left = 0; }
            else { TAKE(i); i++; wins_left++; wins_right = 0; }
            continue;
        }
        /* galloping mode */
        for (;;) {
            uint64_t c = gallop_count(A, i, mid, A->key + j * ks, 1);
            for (uint64_t t = 0; t < c; t++) { TAKE(i); i++; }
            if (i == mid) break;
            uint64_t d = gallop_count(A, j, hi, A->key + i * ks, 0);
            for (uint64_t t = 0; t < d; t++) { TAKE(j); j++; }
            if (j == hi) break;
            if (c < kGallop && d < kGallop) break;
        }
        wins_left = wins_right = 0;
    }
    while (i < mid) { TAKE(i); i++; }
    while (j < hi) { TAKE(j); j++; }
#undef TAKE
    memcpy(A->key + lo * ks, tk, (hi - lo) * ks);
    if (A->pay) memcpy(A->pay + lo, tp, (hi - lo) * sizeof(uint32_t));
}

static size_t key_size(int type) {
    return (type == ORK_I64 || type == ORK_U64) ? 8 : 4;
}

/* State of Alg. PowerSort: the run stack X (starts and ends), the power stack
 * P, and the current run A[s1..e1).  Both stacks hold at most floor(lg n)+1
 * entries (Sec. 3.2.2); 66 covers every 64-bit n.  With A == NULL only the
 * merge order is computed (no data moves). */
typedef struct {
    uint64_t n;
    uint64_t xs[66], xe[66];
    unsigned ps[66];
    int top;
    uint64_t s1, e1;
    arr_t *A;
    unsigned char *tk;
    uint32_t *tp;
    ora_merge *merges;  /* optional record of merges in execution order */
    int galloping;      /* merge with merge_runs_galloping */
    uint8_t *powers;    /* optional record of boundary powers, left to right */
    uint64_t nm, np, M;
} sched_t;

static void do_merge(sched_t *S, uint64_t lo, uint64_t mid, uint64_t hi) {
    if (S->A) {
        if (S->galloping) merge_runs_galloping(S->A, lo, mid, hi, S->tk, S->tp);
        else merge_runs(S->A, lo, mid, hi, S->tk, S->tp);
    }
    if (S->merges) { S->merges[S->nm].lo = lo; S->merges[S->nm].mid = mid; S->merges[S->nm].hi = hi; }
    S->nm++;
    S->M += hi - lo; /* merge cost of one merge = size of its result (Sec. 2.2) */
}

/* One iteration of the main loop of Alg. PowerSort for the next run
 * A[s2..e2): its node power, the pops-and-merges while the stack top has a
 * larger power, and the push. */
static void next_run(sched_t *S, uint64_t s2, uint64_t e2) {
    unsigned p = node_power(S->s1, S->e1 - S->s1, s2, e2 - s2, S->n);
    if (S->powers) S->powers[S->np] = (uint8_t)p;
    S->np++;
    while (S->top > 0 && S->ps[S->top - 1] > p) {
        S->top--;
        /* the popped run ends where the current run starts */
        do_merge(S, S->xs[S->top], S->s1, S->e1);
        S->s1 = S->xs[S->top];
    }
    S->xs[S->top] = S->s1;
    S->xe[S->top] = S->e1;
    S->ps[S->top] = p;
    S->top++;
    S->s1 = s2;
    S->e1 = e2;
}

/* Final loop of Alg. PowerSort: merge everything left on the stack. */
static void finish(sched_t *S) {
    while (S->top > 0) {
        S->top--;
        do_merge(S, S->xs[S->top], S->s1, S->e1);
        S->s1 = S->xs[S->top];
    }
}

/* Find the run that starts at s and extend it to the minimum run length w
 * (App. B.4): a run shorter than w becomes A[s..min(n, s+w)), sorted by
 * insertion sort with the run as its presorted prefix. */
static uint64_t next_leaf(arr_t *A, uint64_t s, uint64_t n, uint32_t w) {
    uint64_t e = extend_run_right(A, s, n);
    if (e - s < w) {
        uint64_t ew = (s + w < n) ? s + w : n;
        insertion_sort(A, s, ew, e - s);
        e = ew;
    }
    return e;
}

/*
 * Sort keys[0..n) (and payload alongside, if not NULL) in place with
 * powersort and minimum run length w.  Optional outputs (each may be NULL):
 *   starts : r+1 run starts after min-run extension, starts[r] = n
 *            (capacity n+1);
 *   powers : the r-1 boundary powers in left-to-right order (capacity n);
 *   merges : the r-1 merges in execution order (capacity n);
 * r_out receives r, merge_cost_out receives M.  Returns 0, or -1 on bad
 * arguments or allocation failure.
 */
static int powersort_impl(void *keys, uint32_t *payload, uint64_t n, int type, uint32_t w,
                          uint64_t *starts, uint8_t *powers, ora_merge *merges,
                          uint64_t *r_out, uint64_t *merge_cost_out, int galloping) {
    if (type < ORK_I32 || type > ORK_F32 || w < 1) return -1;
    arr_t A = { (unsigned char *)keys, payload, key_size(type), type };
    g_comparisons = 0;
    sched_t S;
    uint64_t r = 0;
    memset(&S, 0, sizeof S);
    if (n == 0) {
        if (starts) starts[0] = 0;
        if (r_out) *r_out = 0;
        if (merge_cost_out) *merge_cost_out = 0;
        return 0;
    }
    S.n = n;
    S.A = &A;
    S.merges = merges;
    S.powers = powers;
    S.galloping = galloping;
    S.tk = (unsigned char *)malloc(n * A.ks);
    S.tp = (uint32_t *)malloc(n * sizeof(uint32_t));
    if (!S.tk || !S.tp) { free(S.tk); free(S.tp); return -1; }

    S.s1 = 0;
    S.e1 = next_leaf(&A, 0, n, w);
    if (starts) starts[r] = 0;
    r++;
    while (S.e1 < n) {
        uint64_t s2 = S.e1;
        uint64_t e2 = next_leaf(&A, s2, n, w);
        if (starts) starts[r] = s2;
        r++;
        next_run(&S, s2, e2);
    }
    finish(&S);
    if (starts) starts[r] = n;
    if (r_out) *r_out = r;
    if (merge_cost_out) *merge_cost_out = S.M;
    free(S.tk);
    free(S.tp);
    return 0;
}

int oracle_powersort(void *keys, uint32_t *payload, uint64_t n, int type, uint32_t w,
                     uint64_t *starts, uint8_t *powers, ora_merge *merges,
                     uint64_t *r_out, uint64_t *merge_cost_out) {
    return powersort_impl(keys, payload, n, type, w, starts, powers, merges, r_out, merge_cost_out, 0);
}

/* oracle_powersort with galloping merges: the same runs, tree, merges, merge
 * cost and result; only the key comparisons differ. */
int oracle_powersort_galloping(void *keys, uint32_t *payload, uint64_t n, int type, uint32_t w,
                               uint64_t *starts, uint8_t *powers, ora_merge *merges,
                               uint64_t *r_out, uint64_t *merge_cost_out) {
    return powersort_impl(keys, payload, n, type, w, starts, powers, merges, r_out, merge_cost_out, 1);
}

/* The merge order of Alg. PowerSort for given run lengths L[0..r) (no data):
 * the same stack discipline as oracle_powersort, fed with the runs
 * [sum L[<i], sum L[<=i]).  Records the r-1 powers and merges and returns M
 * through merge_cost_out.  Returns 0, or -1 if some length is 0. */
int oracle_merge_order(const uint64_t *lengths, uint64_t r, uint8_t *powers, ora_merge *merges,
                       uint64_t *merge_cost_out) {
    sched_t S;
    uint64_t n = 0;
    memset(&S, 0, sizeof S);
    for (uint64_t i = 0; i < r; i++) {
        if (lengths[i] == 0) return -1;
        n += lengths[i];
    }
    if (merge_cost_out) *merge_cost_out = 0;
    if (r == 0) return 0;
    S.n = n;
    S.merges = merges;
    S.powers = powers;
    S.s1 = 0;
    S.e1 = lengths[0];
    for (uint64_t i = 1; i < r; i++) next_run(&S, S.e1, S.e1 + lengths[i]);
    finish(&S);
    if (merge_cost_out) *merge_cost_out = S.M;
    return 0;
}

/* Independent sorts of the segments [offsets[g], offsets[g+1]) of one array;
 * each segment is a whole powersort with its own n and origin.  Per-segment
 * merge costs go to costs[g] (may be NULL); the return value is 0 or -1. */
int oracle_segmented_powersort(void *keys, uint32_t *payload, const uint64_t *offsets,
                               uint64_t nseg, int type, uint32_t w, uint64_t *costs) {
    size_t ks = key_size(type);
    for (uint64_t g = 0; g < nseg; g++) {
        uint64_t a = offsets[g], b = offsets[g + 1];
        uint64_t M = 0;
        if (b < a) return -1;
        int rc = oracle_powersort((unsigned char *)keys + a * ks, payload ? payload + a : NULL,
                                  b - a, type, w, NULL, NULL, NULL, NULL, &M);
        if (rc) return rc;
        if (costs) costs[g] = M;
    }
    return 0;
}

/* The node power of Def. "Node Power" for two adjacent runs, exposed so that
 * the tests can evaluate the defining loop on hand-picked run lengths. */
unsigned oracle_node_power(uint64_t s1, uint64_t n1, uint64_t s2, uint64_t n2, uint64_t n) {
    return node_power(s1, n1, s2, n2, n);
}

/* ------------------------------------------------------------------ peeksort
 *
 * Alg. PeekSort (Sec. 3.1) over the same leaves as above: the runs of the
 * Sec. 2 convention, each extended to the minimum run length w (App. B.4).
 * The recursion sees a range A[l..r] (inclusive, as in the paper) made of
 * whole leaves, whose first leaf is A[l..e] and whose last leaf is A[s..r]:
 *   - a single leaf (e == r) needs nothing;
 *   - with m = l + floor((r - l) / 2): if m <= e, cut after the first leaf;
 *     if m >= s, cut before the last leaf; otherwise take the leaf A[i..j]
 *     that contains m and cut before it if m - i < j - m, else after it;
 *   - sort both sides recursively, then merge them (left run first on ties).
 * So the merges come out in post-order, each charged its result size.
 * Parity status: pinned (Fig. 1's left tree, the bound of Thm. "peeksort",
 * an independent nearest-boundary formulation, stable-sort output).
 */
typedef struct {
    arr_t *A;                 /* NULL: merge order only */
    unsigned char *tk;
    uint32_t *tp;
    const uint64_t *S;        /* leaf starts, S[r] = n */
    ora_merge *merges;        /* optional, post-order */
    uint8_t *depth;           /* optional leaf depths */
    uint64_t nm, M;
} peek_t;

/* Leaf k of [a, b) with S[k] <= x < S[k+1]. */
static uint64_t leaf_containing(const uint64_t *S, uint64_t a, uint64_t b, uint64_t x) {
    uint64_t lo = a, hi = b;  /* invariant: S[lo] <= x < S[hi] */
    while (hi - lo > 1) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (S[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

static void peek_rec(peek_t *P, uint64_t a, uint64_t b, unsigned d) {
    const uint64_t *S = P->S;
    if (b - a < 2) {                        /* one run: already sorted */
        if (P->depth) P->depth[a] = (uint8_t)d;
        return;
    }
    uint64_t l = S[a], r = S[b] - 1;        /* A[l..r] */
    uint64_t e = S[a + 1] - 1;              /* first run A[l..e] */
    uint64_t s = S[b - 1];                  /* last run A[s..r] */
    uint64_t m = l + (r - l) / 2;
    uint64_t cut;                           /* first leaf of the right part */
    if (m <= e) {
        cut = a + 1;
    } else if (m >= s) {
        cut = b - 1;
    } else {
        uint64_t k = leaf_containing(S, a, b, m);
        uint64_t i = S[k], j = S[k + 1] - 1;
        cut = (m - i < j - m) ? k : k + 1;
    }
    peek_rec(P, a, cut, d + 1);
    peek_rec(P, cut, b, d + 1);
    if (P->A) merge_runs(P->A, S[a], S[cut], S[b], P->tk, P->tp);
    if (P->merges) { P->merges[P->nm].lo = S[a]; P->merges[P->nm].mid = S[cut]; P->merges[P->nm].hi = S[b]; }
    P->nm++;
    P->M += S[b] - S[a];
}

/*
 * Sort keys[0..n) (payload alongside, may be NULL) with peeksort and minimum
 * run length w.  Optional outputs: starts (r+1, capacity n+1), merges (r-1 in
 * post-order, capacity n), depth (per leaf, capacity n); r_out, M_out.
 * Returns 0, or -1 on bad arguments or allocation failure.
 */
int oracle_peeksort(void *keys, uint32_t *payload, uint64_t n, int type, uint32_t w, uint64_t *starts,
                    ora_merge *merges, uint8_t *depth, uint64_t *r_out, uint64_t *merge_cost_out) {
    if (type < ORK_I32 || type > ORK_F32 || w < 1) return -1;
    arr_t A = { (unsigned char *)keys, payload, key_size(type), type };
    g_comparisons = 0;
    if (r_out) *r_out = 0;
    if (merge_cost_out) *merge_cost_out = 0;
    if (n == 0) {
        if (starts) starts[0] = 0;
        return 0;
    }
    uint64_t *S = (uint64_t *)malloc((n + 1) * sizeof(uint64_t));
    unsigned char *tk = (unsigned char *)malloc(n * A.ks);
    uint32_t *tp = (uint32_t *)malloc(n * sizeof(uint32_t));
    if (!S || !tk || !tp) { free(S); free(tk); free(tp); return -1; }
    uint64_t r = 0, pos = 0;
    while (pos < n) {                       /* the leaves, left to right */
        S[r++] = pos;
        pos = next_leaf(&A, pos, n, w);
    }
    S[r] = n;
    peek_t P = { &A, tk, tp, S, merges, depth, 0, 0 };
    peek_rec(&P, 0, r, 0);
    if (starts) memcpy(starts, S, (r + 1) * sizeof(uint64_t));
    if (r_out) *r_out = r;
    if (merge_cost_out) *merge_cost_out = P.M;
    free(S);
    free(tk);
    free(tp);
    return 0;
}

/* Peeksort's merge order for given run lengths L[0..r) (no data): records
 * the r-1 merges in post-order and the leaf depths; M via merge_cost_out.
 * Returns 0, or -1 if some length is 0 or memory runs out. */
int oracle_peek_merge_order(const uint64_t *lengths, uint64_t r, ora_merge *merges, uint8_t *depth,
                            uint64_t *merge_cost_out) {
    if (merge_cost_out) *merge_cost_out = 0;
    if (r == 0) return 0;
    uint64_t *S = (uint64_t *)malloc((r + 1) * sizeof(uint64_t));
    if (!S) return -1;
    S[0] = 0;
    for (uint64_t i = 0; i < r; i++) {
        if (lengths[i] == 0) { free(S); return -1; }
        S[i + 1] = S[i] + lengths[i];
    }
    peek_t P = { NULL, NULL, NULL, S, merges, depth, 0, 0 };
    peek_rec(&P, 0, r, 0);
    if (merge_cost_out) *merge_cost_out = P.M;
    free(S);
    return 0;
}

/* Peeksort of every segment [offsets[g], offsets[g+1]) on its own;
 * per-segment merge costs go to costs[g] (may be NULL). */
int oracle_segmented_peeksort(void *keys, uint32_t *payload, const uint64_t *offsets, uint64_t nseg,
                              int type, uint32_t w, uint64_t *costs) {
    size_t ks = key_size(type);
    for (uint64_t g = 0; g < nseg; g++) {
        uint64_t a = offsets[g], b = offsets[g + 1];
        uint64_t M = 0;
        if (b < a) return -1;
        int rc = oracle_peeksort((unsigned char *)keys + a * ks, payload ? payload + a : NULL, b - a, type, w,
                                 NULL, NULL, NULL, NULL, &M);
        if (rc) return rc;
        if (costs) costs[g] = M;
    }
    return 0;
}

/* ---------------------------------------------------- elementary mergesorts
 *
 * The two non-natural mergesorts the paper's experiments compare against
 * (Sec. 4.1, setup): top-down and bottom-up mergesort in Sedgewick's form,
 * each with two changes the paper states: before a merge, check whether its
 * two runs are already in order (the left run's last key not above the right
 * run's first key) and skip the merge if so; and sort small pieces by
 * insertion sort: top-down, every subproblem of at most w elements;
 * bottom-up, the chunks of w elements it starts from.  Both merge with
 * merge_runs above (stable, left run first on ties).  The merge cost counts
 * the result sizes of the merges actually run (Sec. 2.2); insertion sorts are
 * not merges.
 * Parity status: pinned (stable-sort output; M = 0 on sorted input; the
 * closed forms of the non-adaptive recursions on strictly decreasing input,
 * where no check fires; and M recomputed from the original data by the
 * condition "some key of the right part is below some key of the left part"
 * over the fixed recursion shapes).
 */

/* Top-down: A[lo..hi) splits as in Sedgewick's m = (l + r) / 2 on inclusive
 * bounds, so the left half takes the ceiling of half the elements. */
static void topdown_rec(arr_t *A, uint64_t lo, uint64_t hi, uint32_t w, unsigned char *tk, uint32_t *tp,
                        uint64_t *M) {
    if (hi - lo <= w) {
        insertion_sort(A, lo, hi, 0);
        return;
    }
    uint64_t mid = lo + (hi - lo + 1) / 2;
    topdown_rec(A, lo, mid, w, tk, tp, M);
    topdown_rec(A, mid, hi, w, tk, tp, M);
    if (less_at(A, mid, mid - 1)) {  /* not already in order */
        merge_runs(A, lo, mid, hi, tk, tp);
        *M += hi - lo;
    }
}

/* Sort keys[0..n) (payload alongside, may be NULL) by top-down mergesort
 * with cutoff w; merge cost via merge_cost_out.  Returns 0 or -1. */
int oracle_topdown_mergesort(void *keys, uint32_t *payload, uint64_t n, int type, uint32_t w,
                             uint64_t *merge_cost_out) {
    if (type < ORK_I32 || type > ORK_F32 || w < 1) return -1;
    arr_t A = { (unsigned char *)keys, payload, key_size(type), type };
    g_comparisons = 0;
    uint64_t M = 0;
    if (n > 0) {
        unsigned char *tk = (unsigned char *)malloc(n * A.ks);
        uint32_t *tp = (uint32_t *)malloc(n * sizeof(uint32_t));
        if (!tk || !tp) { free(tk); free(tp); return -1; }
        topdown_rec(&A, 0, n, w, tk, tp, &M);
        free(tk);
        free(tp);
    }
    if (merge_cost_out) *merge_cost_out = M;
    return 0;
}

/* Sort keys[0..n) by bottom-up mergesort: insertion-sort the chunks
 * [k w, (k+1) w), then for run length m = w, 2w, 4w, ... merge each pair of
 * neighbouring runs [i, i+m) and [i+m, min(i+2m, n)) for i = 0, 2m, 4m, ...
 * while i + m < n (a last run without a partner stays as it is).  Returns 0
 * or -1. */
int oracle_bottomup_mergesort(void *keys, uint32_t *payload, uint64_t n, int type, uint32_t w,
                              uint64_t *merge_cost_out) {
    if (type < ORK_I32 || type > ORK_F32 || w < 1) return -1;
    arr_t A = { (unsigned char *)keys, payload, key_size(type), type };
    g_comparisons = 0;
    uint64_t M = 0;
    if (n > 0) {
        unsigned char *tk = (unsigned char *)malloc(n * A.ks);
        uint32_t *tp = (uint32_t *)malloc(n * sizeof(uint32_t));
        if (!tk || !tp) { free(tk); free(tp); return -1; }
        for (uint64_t s = 0; s < n; s += w) insertion_sort(&A, s, (s + w < n) ? s + w : n, 0);
        for (uint64_t m = w; m < n; m *= 2) {
            for (uint64_t lo = 0; lo + m < n; lo += 2 * m) {
                uint64_t mid = lo + m, hi = (lo + 2 * m < n) ? lo + 2 * m : n;
                if (less_at(&A, mid, mid - 1)) {
                    merge_runs(&A, lo, mid, hi, tk, tp);
                    M += hi - lo;
                }
            }
        }
        free(tk);
        free(tp);
    }
    if (merge_cost_out) *merge_cost_out = M;
    return 0;
}

/* Key comparisons made by the most recent oracle_powersort,
 * oracle_peeksort or elementary mergesort call on this thread: run
 * detection, min-run insertion sorts and merges. */
uint64_t oracle_last_comparisons(void) {
    return g_comparisons;
}
