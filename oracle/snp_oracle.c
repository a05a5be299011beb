/*
 * Plain CPU oracle for the breadth-first expansion of the computation tree of a
 * spiking neural P system without delays, and of the variant with delays that
 * the paper sets aside (Section 2.1, opening) in the form of the work it cites
 * for SN P systems (stated at delay_step below).
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
 * CPU-baseline leg call this file; the simulator library never links, includes
 * or calls it, and it includes nothing of the library.
 *
 * Everything is single-threaded, written for obviousness, with spike counts
 * held in int64_t and range-checked against the element type's maximum:
 *
 *   - the spiking transition matrix M is built entry by entry from
 *     Definition 2 (Section 2.2);
 *   - a rule with regular expression E = a^i (a^j)* (j = 0: exactly a^i),
 *     consumption c and production p applies to a neuron holding n spikes iff
 *     a^n is in L(E) and n >= c (Section 2.1, rule forms b-1 and b-3);
 *   - the valid spiking vectors of a configuration fire exactly one applicable
 *     rule in every neuron that has one and nothing elsewhere (Section 2.2,
 *     "validity"; Section 2.1, one rule per neuron, all neurons in unison); they
 *     are listed in the order of Algorithm 2 step II-3: neuron 1 is the most
 *     significant position, rules of a neuron in their total order;
 *   - a child is C' = C + S.M (Equation next-config);
 *   - the tree is walked breadth first with one global list of produced
 *     configurations, and a configuration produced before is not expanded again
 *     (Algorithm 1 step IV, second stopping criterion);
 *   - with delays, a step follows the definition of a delayed rule directly
 *     (delay_step), not through M.
 *
 * Readings taken where the paper is silent are stated next to the code that
 * takes them.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Status codes (same integers as the simulator's public header documents). */
#define OR_OK 0
#define OR_ERR_INVALID 1
#define OR_ERR_OVERFLOW 2
#define OR_ERR_CAPACITY 3
#define OR_ERR_NOMEM 5

/* Stop reasons (same integers as the simulator's public header documents). */
#define OR_STOP_EMPTY_FRONTIER 0
#define OR_STOP_ALL_HALTING 1
#define OR_STOP_DEPTH 2
#define OR_STOP_CAP 3
#define OR_STOP_BUDGET 4

typedef struct {
    int32_t m, r, n_syn;
    const int32_t *rule_neuron, *rule_i, *rule_j, *rule_c, *rule_p;
    const int32_t *syn_src, *syn_dst;
    int64_t count_max; /* largest spike count the element type holds */
    const int32_t *rule_d; /* nullable: [r] delay of every rule (NULL: a system without delays) */
} or_system;

/* ------------------------------------------------------------------------- */
/* Definition 2: entry a_{k,n} of the spiking transition matrix.             */
/* a = -c if rule k belongs to neuron n; p if rule k belongs to neuron s != n */
/* and (s, n) is a synapse; 0 otherwise.                                      */
/* ------------------------------------------------------------------------- */
static int has_synapse(const or_system *sys, int32_t s, int32_t d) {
    for (int32_t e = 0; e < sys->n_syn; ++e)
        if (sys->syn_src[e] == s && sys->syn_dst[e] == d) return 1;
    return 0;
}

int or_matrix_dense(const or_system *sys, int64_t *M /* r*m row-major */) {
    for (int32_t k = 0; k < sys->r; ++k) {
        int32_t owner = sys->rule_neuron[k];
        for (int32_t n = 0; n < sys->m; ++n) {
            int64_t a;
            if (n == owner) a = -(int64_t)sys->rule_c[k];
            else if (has_synapse(sys, owner, n)) a = sys->rule_p[k];
            else a = 0;
            M[(int64_t)k * sys->m + n] = a;
        }
    }
    return OR_OK;
}

/* Sparse copy of the nonzero entries of M, row by row (the same Definition 2,
 * gathered per row so that large systems fit in memory). */
typedef struct {
    int64_t *row_ptr; /* r + 1 */
    int32_t *col;
    int64_t *val;
    int32_t *nrule_ptr; /* m + 1: the rules of neuron n are nrule[nrule_ptr[n] .. nrule_ptr[n+1]) */
    int32_t *nrule;     /* rule ids, in the total order */
} or_rows;

static void rows_free(or_rows *R) {
    free(R->row_ptr); free(R->col); free(R->val); free(R->nrule_ptr); free(R->nrule);
    R->row_ptr = NULL; R->col = NULL; R->val = NULL; R->nrule_ptr = NULL; R->nrule = NULL;
}

static int rows_build(const or_system *sys, or_rows *R) {
    /* out-neighbour lists of every neuron, in synapse order */
    int64_t *deg = calloc((size_t)sys->m + 1, sizeof(int64_t));
    int32_t *adj = malloc(sizeof(int32_t) * (size_t)(sys->n_syn > 0 ? sys->n_syn : 1));
    int64_t *fill = calloc((size_t)sys->m + 1, sizeof(int64_t));
    if (!deg || !adj || !fill) { free(deg); free(adj); free(fill); return OR_ERR_NOMEM; }
    for (int32_t e = 0; e < sys->n_syn; ++e) deg[sys->syn_src[e] + 1]++;
    for (int32_t n = 0; n < sys->m; ++n) deg[n + 1] += deg[n];
    for (int32_t e = 0; e < sys->n_syn; ++e) {
        int32_t s = sys->syn_src[e];
        adj[deg[s] + fill[s]++] = sys->syn_dst[e];
    }
    int64_t nnz = 0;
    for (int32_t k = 0; k < sys->r; ++k) {
        int32_t s = sys->rule_neuron[k];
        nnz += 1 + (sys->rule_p[k] != 0 ? deg[s + 1] - deg[s] : 0);
    }
    R->row_ptr = malloc(sizeof(int64_t) * ((size_t)sys->r + 1));
    R->col = malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    R->val = malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
    if (!R->row_ptr || !R->col || !R->val) { free(deg); free(adj); free(fill); rows_free(R); return OR_ERR_NOMEM; }
    int64_t q = 0;
    for (int32_t k = 0; k < sys->r; ++k) {
        int32_t s = sys->rule_neuron[k];
        R->row_ptr[k] = q;
        R->col[q] = s; R->val[q] = -(int64_t)sys->rule_c[k]; ++q;      /* -c on the own neuron */
        if (sys->rule_p[k] != 0)
            for (int64_t e = deg[s]; e < deg[s + 1]; ++e) {            /* p on every synapse target */
                R->col[q] = adj[e]; R->val[q] = sys->rule_p[k]; ++q;
            }
    }
    R->row_ptr[sys->r] = q;
    free(deg); free(adj); free(fill);
    /* rules of every neuron, in the total order */
    R->nrule_ptr = calloc((size_t)sys->m + 1, sizeof(int32_t));
    R->nrule = malloc(sizeof(int32_t) * (size_t)(sys->r > 0 ? sys->r : 1));
    if (!R->nrule_ptr || !R->nrule) { rows_free(R); return OR_ERR_NOMEM; }
    int32_t w = 0;
    for (int32_t n = 0; n < sys->m; ++n) {
        R->nrule_ptr[n] = w;
        for (int32_t k = 0; k < sys->r; ++k)
            if (sys->rule_neuron[k] == n) R->nrule[w++] = k;
    }
    R->nrule_ptr[sys->m] = w;
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Rule applicability (Section 2.1): a^n in L(a^i (a^j)*) and n >= c.         */
/* L(a^i (a^j)*) = { a^(i + t*j) : t >= 0 }; with j = 0 it is { a^i }.        */
/* ------------------------------------------------------------------------- */
int or_applicable(int64_t n, int32_t i, int32_t j, int32_t c) {
    if (n < c) return 0;
    if (n < i) return 0;
    if (j == 0) return n == i;
    return (n - i) % j == 0;
}

/* Rules of neuron n that apply to spike count x, in the total order. */
static int32_t applicable_rules(const or_system *sys, const or_rows *R, int32_t n, int64_t x, int32_t *out) {
    int32_t w = 0;
    for (int32_t q = R->nrule_ptr[n]; q < R->nrule_ptr[n + 1]; ++q) {
        int32_t k = R->nrule[q];
        if (or_applicable(x, sys->rule_i[k], sys->rule_j[k], sys->rule_c[k])) out[w++] = k;
    }
    return w;
}

/* ------------------------------------------------------------------------- */
/* Enumeration of the valid spiking vectors of one configuration, in the      */
/* order of Algorithm 2 step II-3, by nested loops written as an odometer:    */
/* neuron 1 is the outermost loop, the last neuron the innermost, and the     */
/* loop of a neuron runs over its applicable rules in their total order.      */
/* A neuron without an applicable rule fires nothing (its loop has one pass). */
/* ------------------------------------------------------------------------- */
typedef struct {
    const or_system *sys;
    int32_t *start;   /* m+1 offsets into app */
    int32_t *app;     /* applicable rules, neuron by neuron */
    int32_t *digit;   /* current position of every neuron's loop */
    int32_t any;      /* some neuron has an applicable rule */
    int32_t waiting;  /* with delays: some neuron is closed or about to send (wait >= 1) */
    int32_t done;
} or_enum;

/* wait (nullable, m entries): with delays, the steps neuron n still waits
 * before it sends its pending spikes (0: open).  A waiting neuron applies no
 * rule.  A configuration has children when some neuron has an applicable rule
 * or some neuron waits; when only the latter holds, its one child fires
 * nothing (the countdown still moves). */
static int enum_open(or_enum *E, const or_system *sys, const or_rows *R, const int64_t *C, const int64_t *wait) {
    E->sys = sys;
    E->start = malloc(sizeof(int32_t) * ((size_t)sys->m + 1));
    E->app = malloc(sizeof(int32_t) * (size_t)(sys->r > 0 ? sys->r : 1));
    E->digit = calloc((size_t)sys->m + 1, sizeof(int32_t));
    if (!E->start || !E->app || !E->digit) return OR_ERR_NOMEM;
    int32_t q = 0;
    E->any = 0;
    E->waiting = 0;
    for (int32_t n = 0; n < sys->m; ++n) {
        E->start[n] = q;
        if (wait && wait[n] >= 1) {
            E->waiting = 1;
            continue;
        }
        q += applicable_rules(sys, R, n, C[n], E->app + q);
        if (q > E->start[n]) E->any = 1;
    }
    E->start[sys->m] = q;
    E->done = !E->any && !E->waiting; /* no applicable rule and nothing pending: halting, no child */
    return OR_OK;
}

static void enum_close(or_enum *E) { free(E->start); free(E->app); free(E->digit); }

static int32_t enum_width(const or_enum *E, int32_t n) { return E->start[n + 1] - E->start[n]; }

/* The spiking vector at the odometer position, written as 0/1 over the r rules. */
static void enum_spiking_vector(const or_enum *E, uint8_t *S) {
    memset(S, 0, (size_t)E->sys->r);
    for (int32_t n = 0; n < E->sys->m; ++n)
        if (enum_width(E, n) > 0) S[E->app[E->start[n] + E->digit[n]]] = 1;
}

/* Advance to the next spiking vector; the innermost (last) neuron moves first. */
static void enum_next(or_enum *E) {
    for (int32_t n = E->sys->m - 1; n >= 0; --n) {
        int32_t w = enum_width(E, n);
        if (w <= 1) continue;
        if (++E->digit[n] < w) return;
        E->digit[n] = 0;
    }
    E->done = 1;
}

/* Equation (next-config): C' = C + S.M, entry by entry, over the nonzeros of the
 * fired rows.  Returns OR_ERR_OVERFLOW when an entry leaves [0, count_max]. */
static int next_config(const or_system *sys, const or_rows *R, const int64_t *C, const uint8_t *S, int64_t *out) {
    for (int32_t n = 0; n < sys->m; ++n) out[n] = C[n];
    for (int32_t k = 0; k < sys->r; ++k) {
        if (!S[k]) continue;
        for (int64_t q = R->row_ptr[k]; q < R->row_ptr[k + 1]; ++q) out[R->col[q]] += R->val[q];
    }
    for (int32_t n = 0; n < sys->m; ++n)
        if (out[n] < 0 || out[n] > sys->count_max) return OR_ERR_OVERFLOW;
    return OR_OK;
}

/* All children of C in order (at most max_out are written).  *psi receives the
 * number of valid spiking vectors, saturated at max_count_psi; 0 when halting.
 * S_out (nullable) receives the spiking vectors as 0/1 bytes, r per child. */
int or_children(const or_system *sys, const int64_t *C, int64_t max_out, int64_t *out_rows,
                uint8_t *S_out, int64_t *psi) {
    if (sys->rule_d) return OR_ERR_INVALID; /* rows with delays carry more entries: or_bfs only */
    or_rows R = {0};
    or_enum E = {0};
    int st = rows_build(sys, &R);
    if (st) return st;
    st = enum_open(&E, sys, &R, C, NULL);
    uint8_t *S = malloc((size_t)(sys->r > 0 ? sys->r : 1));
    int64_t *tmp = malloc(sizeof(int64_t) * (size_t)sys->m);
    if (st || !S || !tmp) { rows_free(&R); enum_close(&E); free(S); free(tmp); return OR_ERR_NOMEM; }
    int64_t count = 0;
    while (!E.done) {
        enum_spiking_vector(&E, S);
        if (count < max_out) {
            st = next_config(sys, &R, C, S, tmp);
            if (st) break;
            memcpy(out_rows + count * sys->m, tmp, sizeof(int64_t) * (size_t)sys->m);
            if (S_out) memcpy(S_out + count * sys->r, S, (size_t)sys->r);
        }
        ++count;
        enum_next(&E);
    }
    *psi = count;
    rows_free(&R); enum_close(&E); free(S); free(tmp);
    return st;
}

/* The child of C with index t in Algorithm 2 order (the odometer advanced t
 * times).  Returns OR_ERR_INVALID when C has fewer than t + 1 children. */
int or_child_at(const or_system *sys, const int64_t *C, int64_t t, int64_t *out_row) {
    if (sys->rule_d) return OR_ERR_INVALID; /* rows with delays carry more entries: or_bfs only */
    or_rows R = {0};
    or_enum E = {0};
    int st = rows_build(sys, &R);
    if (st) return st;
    st = enum_open(&E, sys, &R, C, NULL);
    uint8_t *S = malloc((size_t)(sys->r > 0 ? sys->r : 1));
    if (st || !S) { rows_free(&R); enum_close(&E); free(S); return OR_ERR_NOMEM; }
    for (int64_t q = 0; q < t && !E.done; ++q) enum_next(&E);
    if (E.done) st = OR_ERR_INVALID;
    else {
        enum_spiking_vector(&E, S);
        st = next_config(sys, &R, C, S, out_row);
    }
    rows_free(&R); enum_close(&E); free(S);
    return st;
}

/* ------------------------------------------------------------------------- */
/* A set of configurations keyed by the whole vector (the list allGenCk of    */
/* Section 5, used for the membership test of the second stopping criterion). */
/* Open addressing over row indices; FNV-1a over the values picks the slot.   */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t *slot; /* row index or -1 */
    int64_t cap, used;
    int32_t m;
    const int64_t *const *rows; /* rows are looked up through *rows (it may move) */
} or_set;

static uint64_t row_hash(const int64_t *v, int32_t m) {
    uint64_t h = 1469598103934665603ULL;
    const unsigned char *b = (const unsigned char *)v;
    for (size_t q = 0; q < (size_t)m * sizeof(int64_t); ++q) { h ^= b[q]; h *= 1099511628211ULL; }
    return h;
}

static int set_init(or_set *H, int32_t m, const int64_t *const *rows) {
    H->cap = 1024; H->used = 0; H->m = m; H->rows = rows;
    H->slot = malloc(sizeof(int64_t) * (size_t)H->cap);
    if (!H->slot) return OR_ERR_NOMEM;
    for (int64_t q = 0; q < H->cap; ++q) H->slot[q] = -1;
    return OR_OK;
}

static int64_t set_find(const or_set *H, const int64_t *v) {
    uint64_t q = row_hash(v, H->m) & (uint64_t)(H->cap - 1);
    for (;;) {
        int64_t id = H->slot[q];
        if (id < 0) return -1;
        if (memcmp(*H->rows + id * H->m, v, sizeof(int64_t) * (size_t)H->m) == 0) return id;
        q = (q + 1) & (uint64_t)(H->cap - 1);
    }
}

static int set_insert(or_set *H, int64_t id) {
    if (2 * (H->used + 1) > H->cap) {
        int64_t ncap = H->cap * 2;
        int64_t *ns = malloc(sizeof(int64_t) * (size_t)ncap);
        if (!ns) return OR_ERR_NOMEM;
        for (int64_t q = 0; q < ncap; ++q) ns[q] = -1;
        for (int64_t q = 0; q < H->cap; ++q) {
            int64_t x = H->slot[q];
            if (x < 0) continue;
            uint64_t s = row_hash(*H->rows + x * H->m, H->m) & (uint64_t)(ncap - 1);
            while (ns[s] >= 0) s = (s + 1) & (uint64_t)(ncap - 1);
            ns[s] = x;
        }
        free(H->slot); H->slot = ns; H->cap = ncap;
    }
    uint64_t q = row_hash(*H->rows + id * H->m, H->m) & (uint64_t)(H->cap - 1);
    while (H->slot[q] >= 0) q = (q + 1) & (uint64_t)(H->cap - 1);
    H->slot[q] = id;
    H->used++;
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 1: breadth-first walk of the computation tree from C0.           */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t max_depth;        /* < 0: no depth limit */
    int32_t stop_at_cap;      /* nonzero: a level that reaches frontier_cap ends the walk */
    int64_t frontier_cap;     /* <= 0: none.  A level keeps its first frontier_cap new configurations */
    int64_t child_budget;     /* <= 0: none.  At most this many children are enumerated per level */
    int64_t expand_max_count; /* < 0: none.  A configuration holding more spikes than this in some
                                 neuron is recorded but not expanded */
    int32_t first_only;       /* nonzero: only the first valid spiking vector of every configuration
                                 (each neuron fires its first applicable rule): one branch */
    int32_t out_neuron;       /* > 0: neuron out_neuron (1-based) is the output neuron, and every row
                                 carries two more entries after the m counts: the spikes sent to the
                                 environment so far (at most 2 counted) and the steps from the first
                                 of them to the second (see out_track) */
} or_bfs_opts;

/* The output neuron's spike train (Definition 1: out, whose spikes go to the
 * environment; Section 2.1: the number a computation generates is the time
 * between the first two spikes the output neuron sends out).  A row's two
 * extra entries (env, el) follow the train: q spikes leave at a step when the
 * output neuron sends q (without delays: when it fires a rule producing q; 0
 * when it fires nothing), and
 *   env 0: env = min(2, q), el = 0;
 *   env 1: env = min(2, 1 + q), el = el + 1;
 *   env 2: unchanged (el is the number generated).
 * A row with env = 2 is recorded but not expanded: what follows cannot change
 * the number it generated. */
static void out_track(int64_t q, int32_t m, const int64_t *C, int64_t *child) {
    const int64_t env = C[m], el = C[m + 1];
    if (env == 0) {
        child[m] = q < 2 ? q : 2;
        child[m + 1] = 0;
    } else if (env == 1) {
        child[m] = 1 + q < 2 ? 1 + q : 2;
        child[m + 1] = el + 1;
    } else {
        child[m] = env;
        child[m + 1] = el;
    }
}

/* ------------------------------------------------------------------------- */
/* Delays.  The paper treats systems without delays only and points to the  */
/* work it cites for the variant; this is that variant.  A rule              */
/* E/a^c -> a^p; d with d >= 1 used at step s takes its c spikes at once;    */
/* the neuron is then closed at steps s .. s+d-1 (it applies no rule, and    */
/* spikes sent to it at those steps are lost), at step s+d it sends its p    */
/* spikes along its synapses and is open again (it keeps the spikes it gets   */
/* at that step, and applies no rule at it), and from step s+d+1 on it        */
/* applies rules as before.  d = 0 is the step without delays.               */
/*                                                                           */
/* Readings: a neuron sending its delayed spikes at step s+d applies no rule  */
/* at that step (its rule use spans steps s .. s+d, as a rule without delay   */
/* spans its one step); the output neuron's spikes reach the environment at   */
/* the step they are sent, whether the neuron is open or not.                */
/*                                                                           */
/* A configuration holds, besides the spike counts, the state of every       */
/* neuron that owns a rule with d >= 1 ("delayed neuron"): wait, the steps    */
/* until it sends (0: open), and pend, the spikes it will send.  A row is     */
/* the m counts, then the output neuron's two entries (when followed), then   */
/* (wait, pend) of every delayed neuron in neuron order.                     */
/* ------------------------------------------------------------------------- */
static int32_t rule_delay(const or_system *sys, int32_t k) { return sys->rule_d ? sys->rule_d[k] : 0; }

/* col[n] = column of delayed neuron n's wait entry (pend follows it), -1 for
 * the other neurons; the columns start at `first`.  Returns the row width. */
static int32_t delay_columns(const or_system *sys, int32_t first, int32_t *col) {
    int32_t w = first;
    for (int32_t n = 0; n < sys->m; ++n) {
        int delayed = 0;
        for (int32_t k = 0; k < sys->r; ++k)
            if (sys->rule_neuron[k] == n && rule_delay(sys, k) >= 1) delayed = 1;
        col[n] = delayed ? w : -1;
        if (delayed) w += 2;
    }
    return w;
}

/* Entries per row of a walk: m counts, 2 with an output neuron, 2 per delayed neuron. */
int32_t or_row_width(const or_system *sys, int32_t out_neuron) {
    int32_t *col = malloc(sizeof(int32_t) * (size_t)(sys->m > 0 ? sys->m : 1));
    if (!col) return -1;
    int32_t w = delay_columns(sys, sys->m + (out_neuron > 0 ? 2 : 0), col);
    free(col);
    return w;
}

/* One step with delays from row C under the spiking vector S (0/1 over the
 * rules; waiting neurons fire nothing), into `child` (w entries; entries
 * other than the counts and the delay states are copied from C).  emit
 * receives the spikes every neuron sends at this step.  Returns
 * OR_ERR_OVERFLOW when a count leaves [0, count_max]. */
static int delay_step(const or_system *sys, const int32_t *col, int32_t w, const int64_t *C, const uint8_t *S,
                      int64_t *emit, int32_t *fired, int64_t *child) {
    const int32_t m = sys->m;
    for (int32_t n = 0; n < m; ++n) fired[n] = -1;
    for (int32_t k = 0; k < sys->r; ++k)
        if (S[k]) fired[sys->rule_neuron[k]] = k;
    memcpy(child, C, sizeof(int64_t) * (size_t)w);
    /* spikes sent at this step: a rule without delay fired now, or the pending
     * spikes of a neuron whose wait ends now */
    for (int32_t n = 0; n < m; ++n) {
        const int32_t k = fired[n];
        const int64_t wait = col[n] >= 0 ? C[col[n]] : 0;
        if (k >= 0 && rule_delay(sys, k) == 0) emit[n] = sys->rule_p[k];
        else if (wait == 1) emit[n] = C[col[n] + 1];
        else emit[n] = 0;
    }
    /* consumption, then delivery to the neurons open at this step */
    for (int32_t n = 0; n < m; ++n)
        if (fired[n] >= 0) child[n] -= sys->rule_c[fired[n]];
    for (int32_t e = 0; e < sys->n_syn; ++e) {
        const int32_t src = sys->syn_src[e], dst = sys->syn_dst[e];
        const int32_t k = fired[dst];
        const int64_t wait = col[dst] >= 0 ? C[col[dst]] : 0;
        const int closed = (k >= 0 && rule_delay(sys, k) >= 1) || wait >= 2;
        if (!closed) child[dst] += emit[src];
    }
    /* the delayed neurons' new state */
    for (int32_t n = 0; n < m; ++n) {
        if (col[n] < 0) continue;
        const int32_t k = fired[n];
        const int64_t wait = C[col[n]], pend = C[col[n] + 1];
        if (k >= 0 && rule_delay(sys, k) >= 1) {
            child[col[n]] = rule_delay(sys, k);
            child[col[n] + 1] = sys->rule_p[k];
        } else {
            child[col[n]] = wait >= 1 ? wait - 1 : 0;
            child[col[n] + 1] = wait >= 2 ? pend : 0;
        }
    }
    for (int32_t n = 0; n < m; ++n)
        if (child[n] < 0 || child[n] > sys->count_max) return OR_ERR_OVERFLOW;
    return OR_OK;
}

typedef struct {
    /* caller-owned outputs */
    int64_t *rows;        /* rows_cap rows of or_row_width entries (m, + 2 with an output neuron,
                             + 2 per delayed neuron) */
    int64_t rows_cap;
    int64_t *parent;      /* nullable, rows_cap: global index of the parent (-1 for C0) */
    int64_t *tindex;      /* nullable, rows_cap: index of the spiking vector among the parent's */
    int64_t *level_sizes; /* max_levels */
    int64_t *enumerated;  /* nullable, max_levels: children considered when expanding level k */
    int64_t *halting;     /* nullable, max_levels: parents of level k with no child (no applicable
                             rule, and with delays no neuron waiting) */
    int32_t max_levels;
    /* results */
    int32_t n_levels;
    int32_t stop_reason;
    int32_t pad_;
    int64_t n_configs;
} or_bfs_result;

int or_bfs(const or_system *sys, const int64_t *c0, const or_bfs_opts *opt, or_bfs_result *res) {
    const int32_t m = sys->m;
    const int32_t out = opt->out_neuron;
    if (out < 0 || out > m) return OR_ERR_INVALID;
    int32_t *col = malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    if (!col) return OR_ERR_NOMEM;
    const int32_t w = delay_columns(sys, m + (out > 0 ? 2 : 0), col); /* entries per row */
    int st = OR_OK;
    for (int32_t n = 0; n < w; ++n)
        if (c0[n] < 0 || c0[n] > sys->count_max) { free(col); return OR_ERR_OVERFLOW; }
    if (res->rows_cap < 1 || res->max_levels < 1) { free(col); return OR_ERR_CAPACITY; }
    or_rows R = {0};
    if ((st = rows_build(sys, &R))) { free(col); return st; }
    uint8_t *S = malloc((size_t)(sys->r > 0 ? sys->r : 1));
    int64_t *child = malloc(sizeof(int64_t) * (size_t)w);
    int64_t *wait = calloc((size_t)(m > 0 ? m : 1), sizeof(int64_t));
    int64_t *emit = malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    int32_t *fired = malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    const int64_t *rows_view = res->rows;
    or_set H;
    if (!S || !child || !wait || !emit || !fired || set_init(&H, w, &rows_view)) {
        rows_free(&R); free(S); free(child); free(wait); free(emit); free(fired); free(col);
        return OR_ERR_NOMEM;
    }

    /* level 0 = { C0 } */
    memcpy(res->rows, c0, sizeof(int64_t) * (size_t)w);
    if (res->parent) res->parent[0] = -1;
    if (res->tindex) res->tindex[0] = -1;
    int64_t total = 1;
    set_insert(&H, 0);
    res->level_sizes[0] = 1;
    for (int32_t q = 0; q < res->max_levels; ++q) {
        if (res->enumerated) res->enumerated[q] = 0;
        if (res->halting) res->halting[q] = 0;
    }
    int32_t levels = 1;
    int64_t lvl_begin = 0, lvl_end = 1;
    int32_t stop = OR_STOP_DEPTH;

    for (;;) {
        int32_t depth = levels - 1;
        if (opt->max_depth >= 0 && depth >= opt->max_depth) { stop = OR_STOP_DEPTH; break; }
        if (levels >= res->max_levels) { st = OR_ERR_CAPACITY; break; }
        int64_t enumerated = 0, halting = 0, added = 0, last_par = -1;
        int all_halting = 1, budget_hit = 0, cap_hit = 0;
        for (int64_t par = lvl_begin; par < lvl_end && !cap_hit && !budget_hit && st == OR_OK; ++par) {
            const int64_t *C = res->rows + par * w;
            for (int32_t n = 0; n < m; ++n) wait[n] = col[n] >= 0 ? C[col[n]] : 0;
            or_enum E;
            if (enum_open(&E, sys, &R, C, wait)) { enum_close(&E); st = OR_ERR_NOMEM; break; }
            if (E.done) { enum_close(&E); continue; } /* halting: no child */
            all_halting = 0;
            int expand = 1;
            if (opt->expand_max_count >= 0)
                for (int32_t n = 0; n < m; ++n)
                    if (C[n] > opt->expand_max_count) expand = 0;
            if (out > 0 && C[m] >= 2) expand = 0; /* its number is generated */
            int64_t t = 0;
            while (expand && !E.done) {
                if (opt->child_budget > 0 && enumerated >= opt->child_budget) { budget_hit = 1; break; }
                enum_spiking_vector(&E, S);
                int64_t q = 0; /* spikes the output neuron sends at this step */
                if (sys->rule_d) {
                    if ((st = delay_step(sys, col, w, C, S, emit, fired, child))) break;
                    if (out > 0) q = emit[out - 1];
                } else {
                    if ((st = next_config(sys, &R, C, S, child))) break;
                    for (int32_t k = 0; k < sys->r; ++k)
                        if (S[k] && sys->rule_neuron[k] == out - 1) q = sys->rule_p[k];
                }
                if (out > 0) {
                    out_track(q, m, C, child);
                    if (child[m + 1] > sys->count_max) { st = OR_ERR_OVERFLOW; break; }
                }
                ++enumerated;
                last_par = par;
                if (set_find(&H, child) < 0) {
                    if (total >= res->rows_cap) { st = OR_ERR_CAPACITY; break; }
                    memcpy(res->rows + total * w, child, sizeof(int64_t) * (size_t)w);
                    if (res->parent) res->parent[total] = par;
                    if (res->tindex) res->tindex[total] = t;
                    if ((st = set_insert(&H, total))) break;
                    ++total; ++added;
                    if (opt->frontier_cap > 0 && added >= opt->frontier_cap) { cap_hit = 1; break; }
                }
                ++t;
                if (opt->first_only) break; /* the single branch: Algorithm 2's first vector only */
                enum_next(&E);
            }
            /* A budget that runs out exactly at the end of a parent is only "hit" when a
             * later parent of the level still has a child: the check above, made before
             * each child, sees that on the later parent's first child. */
            enum_close(&E);
        }
        if (st) break;
        /* halting parents are counted up to the parent of the last child the
         * level enumerated (all parents when the level was not cut short) */
        const int64_t p_end = (cap_hit || budget_hit) ? last_par + 1 : lvl_end;
        for (int64_t par = lvl_begin; par < p_end; ++par) {
            const int64_t *C = res->rows + par * w;
            for (int32_t n = 0; n < m; ++n) wait[n] = col[n] >= 0 ? C[col[n]] : 0;
            or_enum E;
            if (enum_open(&E, sys, &R, C, wait)) { enum_close(&E); st = OR_ERR_NOMEM; break; }
            if (E.done) halting++;
            enum_close(&E);
        }
        if (st) break;
        if (res->enumerated) res->enumerated[depth] = enumerated;
        if (res->halting) res->halting[depth] = halting;
        if (added > 0) { /* an expansion that produced nothing adds no level */
            res->level_sizes[levels] = added;
            ++levels;
            lvl_begin = lvl_end;
            lvl_end = total;
        }
        if (all_halting) { stop = OR_STOP_ALL_HALTING; break; }
        if (cap_hit && opt->stop_at_cap) { stop = OR_STOP_CAP; break; }
        if (budget_hit) { stop = OR_STOP_BUDGET; break; }
        if (added == 0) { stop = OR_STOP_EMPTY_FRONTIER; break; }
    }
    res->n_levels = levels;
    res->n_configs = total;
    res->stop_reason = stop;
    free(H.slot); rows_free(&R); free(S); free(child); free(wait); free(emit); free(fired); free(col);
    return st;
}

/* ------------------------------------------------------------------------- */
/* Deterministic trajectory: at every step each neuron fires the first of its */
/* applicable rules in the total order (a single branch of the tree the paper */
/* explores), C_{k+1} = C_k + S_k.M.  The run stops early when no rule        */
/* applies (halting).                                                        */
/*                                                                           */
/* Checksum of a trajectory (a test device, not a quantity of the paper):     */
/*   R_n    = mix64((n + 1) * gamma)            (the SplitMix64 stream, seed 0) */
/*   H(C)   = sum over neurons n of (uint32)C[n] * R_n        (mod 2^64)      */
/*   digest = sum over computed steps k (C_0 included) of                     */
/*            mix64(H(C_k) + k * gamma)                          (mod 2^64)   */
/* with mix64 the SplitMix64 output finaliser (Steele, Lea, Flood 2014) and   */
/* gamma = 0x9E3779B97F4A7C15.                                               */
/* first_repeat = least k with C_k equal to some C_l, l < k (-1: none).      */
/* ------------------------------------------------------------------------- */
#define OR_GAMMA 0x9E3779B97F4A7C15ULL

static uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t or_mix64(uint64_t z) { return mix64(z); }

uint64_t or_config_hash(const int64_t *C, int32_t m) {
    uint64_t h = 0;
    for (int32_t n = 0; n < m; ++n) h += (uint64_t)(uint32_t)C[n] * mix64((uint64_t)(n + 1) * OR_GAMMA);
    return h;
}

static uint64_t step_digest(int64_t k, const int64_t *C, int32_t m) {
    return mix64(or_config_hash(C, m) + (uint64_t)k * OR_GAMMA);
}

int or_deterministic(const or_system *sys, const int64_t *c0, int32_t steps, int64_t *final_c,
                     int32_t *halt_step, int32_t *first_repeat, int32_t *steps_done, uint64_t *digest) {
    const int32_t m = sys->m;
    if (sys->rule_d) return OR_ERR_INVALID; /* the trajectory checksum is defined without delays */
    for (int32_t n = 0; n < m; ++n)
        if (c0[n] < 0 || c0[n] > sys->count_max) return OR_ERR_OVERFLOW;
    or_rows R = {0};
    int st = rows_build(sys, &R);
    if (st) return st;
    int64_t hist_cap = (int64_t)steps + 1;
    int64_t *hist = malloc(sizeof(int64_t) * (size_t)hist_cap * (size_t)m);
    uint8_t *S = malloc((size_t)(sys->r > 0 ? sys->r : 1));
    int32_t *app = malloc(sizeof(int32_t) * (size_t)(sys->r > 0 ? sys->r : 1));
    const int64_t *hist_view = hist;
    or_set H;
    if (!hist || !S || !app || set_init(&H, m, &hist_view)) { rows_free(&R); free(hist); free(S); free(app); return OR_ERR_NOMEM; }

    memcpy(hist, c0, sizeof(int64_t) * (size_t)m);
    set_insert(&H, 0);
    uint64_t dg = step_digest(0, hist, m);
    int32_t hstep = -1, frep = -1, k = 0;
    for (k = 0; k < steps; ++k) {
        const int64_t *C = hist + (int64_t)k * m;
        memset(S, 0, (size_t)sys->r);
        int fired = 0;
        for (int32_t n = 0; n < m; ++n) {
            int32_t w = applicable_rules(sys, &R, n, C[n], app);
            if (w > 0) { S[app[0]] = 1; fired = 1; }
        }
        if (!fired) { hstep = k; break; }
        int64_t *Cn = hist + (int64_t)(k + 1) * m;
        if ((st = next_config(sys, &R, C, S, Cn))) break;
        dg += step_digest(k + 1, Cn, m);
        if (frep < 0) {
            if (set_find(&H, Cn) >= 0) frep = k + 1;
            else if ((st = set_insert(&H, k + 1))) break;
        }
    }
    if (st == OR_OK) {
        memcpy(final_c, hist + (int64_t)k * m, sizeof(int64_t) * (size_t)m);
        *halt_step = hstep;
        *first_repeat = frep;
        *steps_done = k;
        *digest = dg;
    }
    free(H.slot); rows_free(&R); free(hist); free(S); free(app);
    return st;
}
