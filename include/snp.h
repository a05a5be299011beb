/*
 * snp.h -- C ABI of libsnp, a gfx950 (MI355X) simulator for spiking neural P
 * systems without delays that expands the computation tree breadth first.
 *
 * Model (Cabarle, Adorna, Martinez-del-Amor, "Simulating Spiking Neural P
 * systems without delays using GPUs", arXiv:1104.1824):
 *   - A system Pi has m neurons and r rules in a total order, grouped neuron by
 *     neuron (Definition 1; Section 2.2 "a total ordering of rules").
 *   - Rule k of neuron s has regular expression E = a^i (a^j)* (j = 0: exactly
 *     a^i), consumes c >= 1 spikes and sends p >= 0 spikes along every synapse
 *     (s, d) (Definition 1 rule forms b-1, b-2, b-3; Definition 2).  It applies
 *     to a neuron holding n spikes iff a^n is in L(E) and n >= c (Section 2.1).
 *   - A configuration C is the vector of spike counts (Section 2.2).  A valid
 *     spiking vector S fires exactly one applicable rule in every neuron that
 *     has one, and nothing in the others (Section 2.2, "validity").
 *   - The next configuration is C' = C + S . M_Pi (Equation next-config) with
 *     M_Pi the r x m spiking transition matrix of Definition 2.
 *   - Breadth-first expansion (Algorithm 1): every valid S of every frontier
 *     configuration is applied; a configuration produced before, at any level,
 *     is not recorded again (Algorithm 1 step IV, second stopping criterion).
 *
 * Canonical order.  The children of one configuration are numbered
 * t = 0 .. Psi-1 in the order of Algorithm 2 step II-3: neuron 1 is the most
 * significant digit, the last neuron the least, and the digit of a neuron
 * selects among its applicable rules in their total order.  A neuron with no
 * applicable rule has one digit value (it fires nothing).  Psi is the product
 * of max(1, omega_n) over neurons (omega_n = number of applicable rules of
 * neuron n, Algorithm 2 II-1/II-2); a configuration where no rule applies
 * anywhere is halting and has Psi = 0.  The children of a frontier are
 * numbered g = 0, 1, ... parent by parent, in frontier order.  Every level
 * lists its new configurations by increasing g of their first occurrence.
 *
 * All arithmetic is integer.  Spike counts are stored as int32 or uint16
 * (snp_count_t); a count outside [0, max of the type] is SNP_ERR_OVERFLOW,
 * never wrapped or saturated.
 *
 * Conventions shared by every entry point:
 *   - Nothing throws across the ABI; every call returns snp_status and, on an
 *     error, snp_last_error() describes it (thread-local, valid until the next
 *     call on the same thread).
 *   - "device pointer" arguments are HIP device memory (e.g. a torch tensor's
 *     data_ptr()); the caller owns them and keeps them alive for the call.
 *     "host pointer" arguments are ordinary CPU memory.
 *   - A row is one configuration: m consecutive elements of the count type.
 *     Arrays of rows are row-major and densely packed.
 *   - A handle is used by one thread at a time and launches all of its work on
 *     the stream given at load (NULL: the default stream).  Every entry point
 *     returns after that stream has finished the call's work.
 *   - Device-side failures (allocation, launch) return SNP_ERR_DEVICE.
 */
#ifndef SNP_H
#define SNP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SNP_OK = 0,
    SNP_ERR_INVALID = 1,  /* malformed system or argument; nothing was changed */
    SNP_ERR_OVERFLOW = 2, /* a spike count left the range of the count type */
    SNP_ERR_CAPACITY = 3, /* an output or internal buffer is too small */
    SNP_ERR_BUDGET = 4,   /* reserved: limits reached are reported as stop reasons */
    SNP_ERR_DEVICE = 5    /* HIP runtime failure */
} snp_status;

typedef enum { SNP_COUNT_I32 = 0, SNP_COUNT_U16 = 1 } snp_count_t;

/* How S . M is evaluated for a chunk of children.  Results are identical. */
typedef enum {
    SNP_PATH_AUTO = 0,   /* per chunk: the int8 matrix-core form when M fits int8 and the chunk's
                            parents have enough canonical children per parent for its segments
                            (one reference pull per run of up to 64 consecutive children of a
                            parent) to cost less than a pull per child; else the sparse form */
    SNP_PATH_SPARSE = 1, /* gather over the in-synapses of every neuron (int32 adds) */
    SNP_PATH_INT8 = 2    /* S (0/1) x M (int8) on MFMA with int32 accumulation; falls back to
                            SPARSE (stats.int8_fallback = 1) when some |M entry| > 127 */
} snp_path;

/* Why a BFS run ended. */
typedef enum {
    SNP_STOP_EMPTY_FRONTIER = 0, /* a level produced no new configuration (second criterion) */
    SNP_STOP_ALL_HALTING = 1,    /* no rule applies in any frontier configuration (first
                                    criterion generalised: the zero vector is halting) */
    SNP_STOP_DEPTH = 2,          /* max_depth levels were expanded */
    SNP_STOP_CAP = 3,            /* a level reached frontier_cap and stop_at_cap was set */
    SNP_STOP_BUDGET = 4          /* child_budget children were enumerated and more remained */
} snp_stop;

/* An SN P system (Definition 1).  All arrays are host pointers and are copied
 * by snp_load / snp_batch_load; the caller keeps ownership. */
typedef struct {
    int32_t m;                  /* neurons, 1 <= m <= 4608 */
    int32_t r;                  /* rules, >= 0 */
    const int32_t *rule_neuron; /* [r] owner neuron (0-based), non-decreasing; <= 16 rules per neuron */
    const int32_t *rule_i;      /* [r] E = a^i (a^j)*: i >= 1 */
    const int32_t *rule_j;      /* [r] j >= 0 (0: E = a^i exactly) */
    const int32_t *rule_c;      /* [r] spikes consumed, 1 <= c <= 65535 */
    const int32_t *rule_p;      /* [r] spikes sent along each out-synapse, 0 <= p <= 65535 */
    int32_t n_syn;              /* synapses, >= 0 */
    const int32_t *syn_src;     /* [n_syn] (src, dst), src != dst, no duplicate pair */
    const int32_t *syn_dst;     /* [n_syn] */
    const int32_t *M;           /* optional [r*m] row-major M_Pi; when non-NULL it must equal
                                   the Definition 2 matrix of the rules and synapses above */
    int32_t count_type;         /* snp_count_t */
    const int32_t *rule_d;      /* optional [r] delays, 0 <= d <= 32767 (NULL: every d = 0).  The paper
                                   treats systems without delays and leaves the variant to the work it
                                   cites (Section 2.1, opening); here a rule E/a^c -> a^p; d with d >= 1
                                   used at step s takes its c spikes at once, its neuron is closed at
                                   steps s .. s+d-1 (it fires nothing, and spikes sent to it then are
                                   lost), and at step s+d it sends its p spikes along its synapses,
                                   keeps the spikes it receives at that step and fires nothing; it
                                   fires again from step s+d+1.  Every neuron owning a rule with d >= 1
                                   adds two entries to a row, after the counts and the output neuron's
                                   spike train, in neuron order: wait (steps until it sends; 0: open)
                                   and pend (the spikes it will send).  A configuration where no rule
                                   applies but some neuron waits has one child (it fires nothing).
                                   With delays a row holds at most 3640 entries, the sparse form runs
                                   every pass (SNP_PATH_INT8 falls back, int8_fallback = 1), and the
                                   batched mode is refused. */
} snp_desc;

typedef struct {
    int32_t path;             /* snp_path */
    int32_t stop_at_cap;      /* nonzero: snp_run ends when a level reaches frontier_cap */
    int64_t frontier_cap;     /* > 0: a level keeps only its first frontier_cap new
                                 configurations (later ones are not recorded as visited);
                                 0: no cap */
    int64_t child_budget;     /* > 0: at most this many children are enumerated per level;
                                 0: no budget */
    int64_t expand_max_count; /* >= 0: a configuration holding more spikes than this in some
                                 neuron is recorded but never expanded; < 0: off */
    int64_t max_rows;         /* > 0: most configurations one run (or one snp_reset and the
                                 snp_expand calls after it) records, C0 included; sizes the
                                 visited set */
    int64_t max_frontier;     /* largest frontier one expansion takes; 0: max_rows */
    int64_t chunk;            /* most children expanded per device pass; 0: automatic */
    uint64_t hash_mask;       /* 0: full 64-bit configuration hash; otherwise the hash is
                                 ANDed with it (forces collisions; results do not change) */
    int32_t profile;          /* 1: time the child expansion kernel with HIP events recorded
                                 on the handle's stream just before and after each launch
                                 (snp_expand_stats.ns_expand); >= 2: time every stage (every
                                 ns_* field); 0: no events.  The events are created for timing
                                 only (no system-scope fence when one is reached). */
    int32_t int8_max_k;       /* int8 path: most rule columns one segment of children may put on
                                 the matrix cores (1..128, values above 64 act as 64; 0: 64); a
                                 segment that needs more is halved until it fits, a single child
                                 being computed by the pull (smaller values force shorter
                                 segments; results do not change) */
    int32_t deterministic;    /* nonzero: every configuration has at most one child, the one
                                 that fires the first applicable rule of every neuron (the first
                                 spiking vector of Algorithm 2 step II-3), so a walk follows a
                                 single branch of the computation tree (Section 2.1: one rule per
                                 neuron, all neurons on a global clock) and ends at its first
                                 repeated configuration (EMPTY_FRONTIER) or at a halting one */
    int32_t out_neuron;       /* > 0: neuron out_neuron (1-based) is the output neuron (Definition 1,
                                 out), and a row holds m + 2 entries: the m counts, then the
                                 output neuron's spike train: the spikes it has sent to the
                                 environment (at most 2 counted) and the steps from the first of
                                 them to the second (0 before the first; after the second, the number
                                 the computation generated, Section 2.1).  q spikes leave at a step
                                 where the output neuron fires a rule producing q; with e spikes
                                 sent and s steps counted before it: e = 0 gives (min(2, q), 0),
                                 e = 1 gives (min(2, 1 + q), s + 1), e = 2 stays.  A configuration
                                 whose train holds 2 spikes is recorded but not expanded.  Runs on
                                 the sparse form (SNP_PATH_INT8 falls back, int8_fallback = 1);
                                 0: off */
    void *stream;             /* hipStream_t for all work of the handle; NULL: default */
    int32_t stage_rows;       /* how snp_run's int8 passes write rows.  Staged: every child's row to
                                 a staging buffer, the commit copying the new ones to the row store.
                                 Keys-first: keys and the visited set first, then the rows, each new
                                 one written once at its place in the row store.  > 0: staged;
                                 < 0: keys-first; 0: keys-first for a pass whose chunk holds at least
                                 64 MiB of rows (where the copy it saves outweighs its two extra
                                 launches), else staged.  A key that met an entry is taken to name the same
                                 configuration until the rows are compared after the row pass; when
                                 two differ (a 32-bit tag or 64-bit key shared by two configurations)
                                 the pass is undone and redone staged (snp_expand_stats.redone), so
                                 results never change.  snp_expand always stages. */
} snp_options;

/* Per-level counters of one expansion. */
typedef struct {
    int64_t parents;         /* frontier configurations */
    int64_t halting_parents; /* parents where no rule applies, counted up to the parent of the last
                                child the level enumerated (all parents when the level was not cut
                                short by frontier_cap or child_budget) */
    int64_t children_total;  /* sum of Psi over the parents examined (a prefix of the frontier
                                large enough for the children enumerated), saturated at 2^62 */
    int64_t enumerated;      /* children in canonical order up to where the level stopped:
                                the cap-filling child, the budget, or all of them */
    int64_t new_configs;     /* configurations recorded for the level */
    int64_t duplicates;      /* enumerated - new_configs: children equal to a configuration
                                recorded before, at this level or an earlier one (Algorithm 1
                                step IV membership test), twins included */
    int64_t expanded;        /* children computed on the device (>= enumerated: the pass that
                                fills the cap runs to its end) */
    int64_t twins;           /* of those, children that fire the later of two twin rules (same
                                neuron, same c and p): they repeat an earlier child, so only
                                their parent and child index are written */
    int64_t collisions;      /* visited-set probes that met an entry with the same 32-bit tag
                                whose full row differed (settled by the row compare) */
    int64_t chunks;          /* device passes used */
    int64_t int8_chunks;     /* of those, passes that ran the int8 matrix-core form (the rest ran
                                the sparse form; SNP_PATH_AUTO picks per pass) */
    int64_t mfma_ops;        /* int8 matrix-core multiply-adds issued by the level, x 2 (one
                                16x16x64 instruction = 32768 integer operations) */
    int32_t truncated;       /* 1: the level reached frontier_cap */
    int32_t budget_hit;      /* 1: child_budget ran out with children left */
    int32_t path_used;       /* snp_path of the last pass (SPARSE or INT8) */
    int32_t int8_fallback;   /* 1: INT8 was requested but M does not fit int8 (or an output neuron
                                is followed, which only the sparse form does) */
    /* Device time of each stage summed over the level's passes, in ns (0 when
     * not timed; see snp_options.profile): applicability + Psi and its prefix
     * sum; child expansion (S.M + C); visited-set insert; first-occurrence flags
     * and their prefix sum; ordered commit. */
    int64_t ns_psi, ns_expand, ns_insert, ns_flags, ns_commit;
    /* In a keys-first pass ns_psi also holds the key pass, the visited-set probe and the flags,
     * ns_expand the row pass, ns_insert the row check, and ns_flags stays 0. */
    int64_t redone;          /* keys-first passes undone and redone staged after their row check */
    int64_t keys_first;      /* passes that ran keys-first (see snp_options.stage_rows) */
} snp_expand_stats;

typedef struct snp_system snp_system; /* opaque; owns derived tables and the visited set */

/* Validate a system, derive M_Pi (Definition 2) and its device tables, and
 * allocate the visited set for opt->max_rows configurations.
 *   desc: host description, copied.  opt: host options, copied (NULL: defaults
 *   with max_rows = 1<<20).  out: receives the handle.
 * Errors: SNP_ERR_INVALID for a malformed system (rule order, i < 1, j < 0,
 * c < 1, p < 0, neuron id out of range, self or duplicate synapse, M that
 * differs from Definition 2, bad count_type or options); SNP_ERR_DEVICE. */
snp_status snp_load(const snp_desc *desc, const snp_options *opt, snp_system **out);

/* Release a handle (NULL is ignored). */
void snp_free(snp_system *sys);

/* Message for the last failed call on this thread ("" if none). */
const char *snp_last_error(void);

/* Number of bytes of one row (m * size of the count type). */
int64_t snp_row_bytes(const snp_system *sys);

/* Start a caller-driven walk (Algorithm 1 step I: the initial configuration
 * becomes the first entry of the list of produced configurations): forget
 * every visited configuration and record C0 (device pointer, one row) as
 * level 0 in the handle's own row store.  The row store (max_rows rows) is
 * allocated on the first call.
 * Errors: SNP_ERR_OVERFLOW if C0 holds a count outside the type's range (only
 * negative counts can be out of range for int32 here). */
snp_status snp_reset(snp_system *sys, const void *c0_dev);

/* Expand one level (Algorithm 1 steps II-III for every frontier configuration).
 *   frontier_dev: device pointer, n rows.  The children of these rows are
 *     enumerated in canonical order and compared with every configuration
 *     recorded since snp_reset (earlier levels and earlier children).
 *   next_dev: device pointer with room for next_capacity rows; receives the new
 *     configurations in first-occurrence order.  *n_next (host) receives their
 *     number.  They are also recorded in the handle as visited.
 *   parent_of_next: nullable device int64 [next_capacity]: index in
 *     frontier_dev of the parent of every new row.
 *   child_of_next: nullable device int64 [next_capacity]: child index t of every
 *     new row within its parent (canonical order).
 *   stats: nullable host pointer, filled on success.
 * frontier_cap, child_budget and expand_max_count of the options apply.
 * Errors: SNP_ERR_CAPACITY when the new rows exceed next_capacity or the
 *   handle's max_rows, or n exceeds max_frontier; *n_next then receives the
 *   number of new rows found so far (a lower bound) and the visited set is left
 *   as it was before the call.  SNP_ERR_OVERFLOW when a child's count leaves
 *   the type's range (the visited set is then left as before the call). */
snp_status snp_expand(snp_system *sys, const void *frontier_dev, int64_t n, void *next_dev,
                      int64_t next_capacity, int64_t *n_next, int64_t *parent_of_next,
                      int64_t *child_of_next, snp_expand_stats *stats);

/* Breadth-first walk from C0 (Algorithm 1) until a stop condition.
 *   c0_dev: device pointer, one row.
 *   max_depth: levels to expand; < 0: no depth limit.
 *   out_dev: device pointer with room for out_capacity rows; receives every
 *     recorded configuration, level after level (level 0 = C0), and serves as
 *     the run's row store (no other copy of the rows is made).
 *   *n_configs (host): rows written.
 *   level_sizes: host int64 [max_levels]: rows of every level; *n_levels (host)
 *     receives the number of levels (an expansion that yields nothing adds none).
 *   *stop_reason (host): snp_stop.
 *   level_stats: nullable host [max_levels]: entries [0, *n_levels) receive the
 *     counters of the expansion of each level (zeros for a level that was not
 *     expanded); later entries are left as they are.
 *   parent_of: nullable device int64 [out_capacity]: row index (in out_dev) of
 *     the parent of every row, -1 for C0.
 *   child_of: nullable device int64 [out_capacity]: child index t of every row
 *     within its parent (canonical order), -1 for C0.
 * Errors: SNP_ERR_CAPACITY when out_capacity, max_levels or max_rows is too
 *   small (rows and levels written so far stay valid and *n_configs, *n_levels
 *   say how many); SNP_ERR_OVERFLOW as for snp_expand, and when C0 holds a
 *   count outside the type's range (C0 is checked on the device together
 *   with the first level, so that level costs no wait of its own; the outputs
 *   are then not meaningful). */
snp_status snp_run(snp_system *sys, const void *c0_dev, int32_t max_depth, void *out_dev,
                   int64_t out_capacity, int64_t *n_configs, int64_t *level_sizes, int32_t max_levels,
                   int32_t *n_levels, int32_t *stop_reason, snp_expand_stats *level_stats,
                   int64_t *parent_of, int64_t *child_of);

/* Launch settings of a handle's walk.  Results never depend on them (only
 * timing does); 0 in a field means the library's built-in choice. */
typedef struct {
    int64_t chunk;       /* canonical children per device pass, 1 .. the handle's chunk
                            (snp_options.chunk or its automatic value: the buffers' size) */
    int32_t int8_tiles;  /* int8 form: consecutive 64-child tiles per workgroup, 0 .. 64 */
    int32_t sparse_run;  /* sparse form (m > 64 or in-degree > 16): consecutive children per
                            wave, 0 .. 1024 */
} snp_tuning;

/* The handle's current settings. */
snp_status snp_get_tuning(const snp_system *sys, snp_tuning *out);

/* Set the handle's settings (host pointer, copied).  Errors: SNP_ERR_INVALID for
 * a field outside its range. */
snp_status snp_set_tuning(snp_system *sys, const snp_tuning *tuning);

/* Autotuner: times whole walks of this workload (snp_run with these arguments,
 * the fastest of three after a warm-up, one for walks above 100 ms) under
 * candidate settings, coordinate by coordinate: chunk = the handle's chunk and
 * its halves down to 1/16 (not under 4096), then int8_tiles in {1, 2, 4, 8, 16}
 * where the int8 form can run, then sparse_run in {4, 8, 16, 32, 64} where the
 * sparse form can run.  The fastest is applied to the handle, returned in
 * *best (nullable) with its walk time in *best_ms (ms, nullable), and, when
 * cache_path (a file name) is non-NULL, recorded there: a JSON object
 * {"snp_tuning_cache": 1, "entries": {key: {"chunk", "int8_tiles",
 * "sparse_run", "ms"}}} whose key names the GPU architecture and hashes the
 * system, the options that shape the walk and max_depth.  Other entries of the
 * file are kept.  out_dev / out_capacity are snp_run's (the rows of the last
 * walk stay there).
 * Errors: those of snp_run; SNP_ERR_INVALID when cache_path exists and is not
 * a tuning cache, or cannot be written. */
snp_status snp_autotune(snp_system *sys, const void *c0_dev, int32_t max_depth, void *out_dev,
                        int64_t out_capacity, const char *cache_path, snp_tuning *best, double *best_ms);

/* Apply the settings recorded in cache_path for this handle's workload (the
 * key snp_autotune uses, with this max_depth), if any: *found (host) = 1 when
 * applied, 0 when the file or the key is missing.
 * Errors: SNP_ERR_INVALID when the file is not a tuning cache. */
snp_status snp_load_tuning(snp_system *sys, const char *cache_path, int32_t max_depth, int32_t *found);

/* ------------------------------------------------------------------------- */
/* Deterministic branch of many independent systems in one launch.            */
/* At every step each neuron fires the first of its applicable rules in the   */
/* total order (the first spiking vector of Algorithm 2; one rule per neuron, */
/* all neurons on a global clock, Section 2.1), C_{k+1} = C_k + S_k . M       */
/* (Equation next-config), until `steps` steps or a configuration where no    */
/* rule applies (halting).                                                   */
/* ------------------------------------------------------------------------- */
typedef struct snp_batch snp_batch; /* opaque; owns the packed tables of all systems */

/* Load n >= 1 systems (host descriptions, copied).  All must share one
 * count_type.  Limits of this mode: m <= 4096, and i, j, c, p <= 255; a
 * launch shape (threads per system, neurons per thread) also needs the
 * largest system to fit one block's 64 KiB of LDS: about
 * 8 r_max + 12 s + 536 w + 1,600 bytes for s = threads x neurons per thread
 * (s >= m_max) and w = threads / 64; shapes that do not fit are skipped.
 * opt: NULL or options; used are `stream`, and `chunk`, which here fixes the
 *   threads per system (256, 512 or 1024; each thread owns up to 4 neurons).
 *   chunk = 0: the first snp_batch_run times every fitting shape on a short
 *   run of the batch and keeps the fastest.  Other fields are ignored.
 * Errors: SNP_ERR_INVALID (as snp_load, plus the limits above, a `chunk`
 *   that does not fit, or no shape that fits), SNP_ERR_DEVICE. */
snp_status snp_batch_load(const snp_desc *descs, int32_t n, const snp_options *opt, snp_batch **out);

void snp_batch_free(snp_batch *b);

/* Element offsets of every system's row in the packed row buffers that
 * snp_batch_run reads and writes: system k occupies elements
 * [offsets[k], offsets[k+1]).  offsets: host int64 [n + 1]. */
snp_status snp_batch_offsets(const snp_batch *b, int64_t *offsets);

/* Launch shape in use: threads per system and neurons per thread (both 0
 * before the first snp_batch_run picks them).  Outputs: host int32. */
snp_status snp_batch_shape(const snp_batch *b, int32_t *threads, int32_t *neurons_per_thread);

/* Run every system from its C0 for at most `steps` steps in one launch.  The
 * launch is recorded once as a HIP graph and replayed while c0_dev,
 * final_dev, steps and detect_repeats stay the same.
 *   c0_dev: device pointer, packed rows (offsets above).
 *   final_dev: device pointer, packed rows: the configuration after the last
 *     computed step (the halting one if the system halted).
 *   halt_step: host int32 [n]: step k whose configuration C_k is halting, -1 if none.
 *   first_repeat: host int32 [n]: least k with C_k equal to an earlier C_l, -1 if
 *     none (or if detect_repeats is 0).
 *   steps_done: host int32 [n]: steps computed.
 *   digest: host uint64 [n]: sum over computed steps k (C_0 included) of
 *     mix64(H(C_k) + k * 0x9E3779B97F4A7C15) mod 2^64, where
 *     H(C) = sum_n (uint32)C[n] * R_n mod 2^64, R_n = mix64((n + 1) * 0x9E3779B97F4A7C15)
 *     and mix64 is the SplitMix64 output finaliser.
 * Errors: SNP_ERR_OVERFLOW when a count leaves the type's range (outputs then
 *   undefined); SNP_ERR_DEVICE when two different configurations of one
 *   trajectory share a 64-bit H, so that repeat detection cannot vouch for
 *   its answer (never observed; the probability is about steps^2 / 2^64). */
snp_status snp_batch_run(snp_batch *b, const void *c0_dev, int32_t steps, int32_t detect_repeats,
                         void *final_dev, int32_t *halt_step, int32_t *first_repeat, int32_t *steps_done,
                         uint64_t *digest);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same run
 * as snp_batch_run, with the same arguments and results, but every scratch
 * buffer of the run (per-system results, checkpoint rows, H sets) lives in
 * one static device array of the library (32 MiB, held by every device the
 * library runs on until the process ends), and the call makes no allocation
 * of any kind: no hipMalloc or hipFree, no HIP graph, no events.  The launch
 * shape is the one an earlier snp_batch_run on this batch picked, else the
 * widest candidate (no timing).
 * Every call on one device shares that device's array: calls that overlap on
 * one device (other threads, other streams) race and must not be made.  The
 * H sets are cleared by a kernel at the start of every call; every other
 * result is written in full by the run.
 * Errors: SNP_ERR_CAPACITY when the run needs more scratch than the array
 *   holds (about (4 + 2 n) x 64 B for n systems, plus steps / 64 + 1
 *   checkpoint rows of every system, plus 12 x 2^ceil(log2(2 steps + 2)) B per
 *   system with repeat detection); otherwise as snp_batch_run. */
snp_status snp_batch_run_static(snp_batch *b, const void *c0_dev, int32_t steps, int32_t detect_repeats,
                                void *final_dev, int32_t *halt_step, int32_t *first_repeat,
                                int32_t *steps_done, uint64_t *digest);

/* Deterministic branch of n systems loaded with snp_load, in one launch
 * (the batched mode above, built from the handles' descriptions on the first
 * call with this list of handles and kept for later calls with the same list).
 *   systems: host array of n handles, all with one count type.
 *   c0_dev: host array of n device pointers, one row each.
 *   steps: most steps per system, 0 <= steps <= 2^24.
 *   final_dev: host array of n device pointers, one row each: the
 *     configuration after the last computed step.
 *   halt_step, first_repeat_step: host int32 [n]; trajectory_digest: host
 *     uint64 [n]; as halt_step, first_repeat and digest of snp_batch_run
 *     (repeat detection on).
 * The batched mode's limits apply (m <= 4096; i, j, c, p <= 255).
 * Errors: SNP_ERR_INVALID (NULL arguments, mixed count types, limits);
 *   SNP_ERR_OVERFLOW; SNP_ERR_DEVICE. */
snp_status snp_run_batch(snp_system *const *systems, int32_t n, const void *const *c0_dev, int32_t steps,
                         void *const *final_dev, int32_t *halt_step, int32_t *first_repeat_step,
                         uint64_t *trajectory_digest);

#ifdef __cplusplus
}
#endif

#endif /* SNP_H */
