// C ABI of libsnp: validation and derivation of a system's tables, the visited
// set, and the host loop over levels and chunks that drives the kernels of
// snp_kernels.hip.  Semantics of every entry point are documented in snp.h.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "snp.h"
#include "snp_handle.hpp"
#include "snp_internal.hpp"

using snp::u64;

namespace {

thread_local std::string g_err;

void set_error_v(const char* fmt, va_list ap) {
    char buf[512];
    vsnprintf(buf, sizeof buf, fmt, ap);
    g_err = buf;
}

snp_status fail(snp_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    set_error_v(fmt, ap);
    va_end(ap);
    return st;
}

}  // namespace

snp_status snp::set_error(snp_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    set_error_v(fmt, ap);
    va_end(ap);
    return st;
}

namespace {

#define HIPCHK(expr)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return fail(SNP_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr int kMaxRulesPerNeuron = 16;  // applicable-rule masks are 16-bit (plus 16 bits of twin marks)
constexpr int kMaxNeurons = 4608;       // per-wave LDS state of the expansion kernel (14 B per neuron) <= 64 KiB
constexpr int kMaxDelayWidth = 3640;    // with delays, 18 B per row entry <= 64 KiB
constexpr int kMaxDelay = 32767;        // a rule's delay (15 bits of the packed fired-rule word)
constexpr long long kInf = LLONG_MAX / 4;

u64 host_mix64(u64 z) {  // SplitMix64 output finaliser
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

u64 next_pow2(u64 x) {
    u64 p = 1;
    while (p < x) p <<= 1;
    return p;
}

template <typename P>
hipError_t dmalloc(P** p, size_t bytes) {
    return hipMalloc((void**)p, bytes > 0 ? bytes : 16);
}

}  // namespace

struct snp_batch {
    int n = 0, elem_bytes = 4, m_max = 0, r_max = 0;
    // launch shape: threads per system and neurons per thread (0: not tuned yet)
    int threads = 0, npt = 0, forced_threads = 0;
    std::vector<std::pair<int, int>> shapes;  // candidates (threads, npt)
    long long count_max = INT_MAX;
    hipStream_t stream = nullptr;
    std::vector<snp::BatchSys> sys;
    std::vector<long long> row_off;  // n + 1
    snp::BatchSys* d_sys = nullptr;
    uint32_t* d_rules = nullptr;
    uint32_t* d_magic = nullptr;
    int *d_nrp = nullptr, *d_in_ptr = nullptr, *d_in_src = nullptr;
    uint32_t *d_fast = nullptr, *d_lut = nullptr;  // tables of the first applicable rule
    int* d_perm = nullptr;                           // slot -> neuron
    uint16_t* d_reg_src = nullptr;                   // per slot: where each pull round reads
    // per-run buffers, grown on demand
    int cap_steps = -1;
    long long ckpt_rows = 0;
    void* d_ckpt = nullptr;
    u64* d_hkey = nullptr;
    int* d_hstep = nullptr;
    u64 table_slots = 0;
    int *d_halt = nullptr, *d_rep = nullptr, *d_done = nullptr;
    u64 *d_digest = nullptr, *d_err = nullptr;
    // the run's launches (fill + kernel) as a graph, replayed while the key matches
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t exec = nullptr;
    struct Key {
        const void *c0, *fin;
        int steps, detect, threads, npt, cap_steps;
        bool operator==(const Key& o) const {
            return c0 == o.c0 && fin == o.fin && steps == o.steps && detect == o.detect && threads == o.threads &&
                   npt == o.npt && cap_steps == o.cap_steps;
        }
    } key{};
    ~snp_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        void* ptrs[] = {d_sys, d_rules, d_magic, d_nrp, d_in_ptr, d_in_src, d_ckpt, d_hkey, d_hstep,
                        d_halt, d_rep, d_done, d_digest, d_err, d_fast, d_lut, d_perm, d_reg_src};
        for (void* p : ptrs)
            if (p) (void)hipFree(p);
    }
};

namespace {

long long row_bytes(const snp_system* S) { return (long long)S->m * S->elem_bytes; }

snp_status validate(const snp_desc* d) {
    if (!d) return fail(SNP_ERR_INVALID, "desc is NULL");
    if (d->m < 1) return fail(SNP_ERR_INVALID, "m must be >= 1 (got %d)", d->m);
    if (d->m > kMaxNeurons) return fail(SNP_ERR_INVALID, "m above %d is not supported", kMaxNeurons);
    if (d->r < 0 || d->n_syn < 0) return fail(SNP_ERR_INVALID, "negative r or n_syn");
    if (d->count_type != SNP_COUNT_I32 && d->count_type != SNP_COUNT_U16)
        return fail(SNP_ERR_INVALID, "count_type must be SNP_COUNT_I32 or SNP_COUNT_U16");
    if (d->r > 0 && (!d->rule_neuron || !d->rule_i || !d->rule_j || !d->rule_c || !d->rule_p))
        return fail(SNP_ERR_INVALID, "rule arrays must be non-NULL when r > 0");
    if (d->n_syn > 0 && (!d->syn_src || !d->syn_dst))
        return fail(SNP_ERR_INVALID, "synapse arrays must be non-NULL when n_syn > 0");
    std::vector<int> per(d->m, 0);
    for (int k = 0; k < d->r; ++k) {
        const int n = d->rule_neuron[k];
        if (n < 0 || n >= d->m) return fail(SNP_ERR_INVALID, "rule %d: neuron %d out of range", k, n);
        if (k > 0 && n < d->rule_neuron[k - 1])
            return fail(SNP_ERR_INVALID, "rule %d: rules must be grouped by non-decreasing neuron", k);
        if (d->rule_i[k] < 1) return fail(SNP_ERR_INVALID, "rule %d: i must be >= 1", k);
        if (d->rule_j[k] < 0) return fail(SNP_ERR_INVALID, "rule %d: j must be >= 0", k);
        if (d->rule_c[k] < 1) return fail(SNP_ERR_INVALID, "rule %d: c must be >= 1", k);
        if (d->rule_p[k] < 0) return fail(SNP_ERR_INVALID, "rule %d: p must be >= 0", k);
        if (d->rule_c[k] > 65535 || d->rule_p[k] > 65535)
            return fail(SNP_ERR_INVALID, "rule %d: c and p must be <= 65535", k);
        if (++per[n] > kMaxRulesPerNeuron)
            return fail(SNP_ERR_INVALID, "neuron %d has more than %d rules", n, kMaxRulesPerNeuron);
        if (d->rule_d && (d->rule_d[k] < 0 || d->rule_d[k] > kMaxDelay))
            return fail(SNP_ERR_INVALID, "rule %d: delay must be in [0, %d]", k, kMaxDelay);
    }
    std::vector<std::pair<int, int>> edges;
    edges.reserve(d->n_syn);
    for (int e = 0; e < d->n_syn; ++e) {
        const int s = d->syn_src[e], t = d->syn_dst[e];
        if (s < 0 || s >= d->m || t < 0 || t >= d->m)
            return fail(SNP_ERR_INVALID, "synapse %d: neuron out of range", e);
        if (s == t) return fail(SNP_ERR_INVALID, "synapse %d: self-synapse (%d,%d)", e, s, t);
        edges.emplace_back(s, t);
    }
    std::sort(edges.begin(), edges.end());
    for (size_t e = 1; e < edges.size(); ++e)
        if (edges[e] == edges[e - 1])
            return fail(SNP_ERR_INVALID, "duplicate synapse (%d,%d)", edges[e].first, edges[e].second);
    return SNP_OK;
}

// Definition 2, entry (k, n) of M_Pi.
int def2_entry(const snp_desc* d, const std::vector<std::vector<char>>& adj, int k, int n) {
    const int owner = d->rule_neuron[k];
    if (n == owner) return -d->rule_c[k];
    if (adj[owner][n]) return d->rule_p[k];
    return 0;
}

// Adds the device time between events a and b to *acc (ns); events are recorded only when profiling.
snp_status add_elapsed(snp_system* S, int a, int b, int64_t* acc) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, S->ev[a], S->ev[b]));
    *acc += (int64_t)((double)ms * 1.0e6);
    return SNP_OK;
}

// Stage marks 0..5; profile 1 records only 1 and 2 (around the expansion kernel).
snp_status mark(snp_system* S, int k) {
    if (S->opt.profile >= 2 || (S->opt.profile == 1 && (k == 1 || k == 2)))
        HIPCHK(hipEventRecord(S->ev[k], S->stream));
    return SNP_OK;
}

snp_status validate_options(const snp_options* o) {
    if (o->path < SNP_PATH_AUTO || o->path > SNP_PATH_INT8) return fail(SNP_ERR_INVALID, "bad path");
    if (o->frontier_cap < 0 || o->child_budget < 0 || o->chunk < 0 || o->max_frontier < 0)
        return fail(SNP_ERR_INVALID, "negative frontier_cap, child_budget, chunk or max_frontier");
    if (o->max_rows < 1 || o->max_rows >= (long long)snp::kStageBase)
        return fail(SNP_ERR_INVALID, "max_rows must be in [1, 2^31)");
    if (o->chunk > (long long)snp::kMaxChunk) return fail(SNP_ERR_INVALID, "chunk above 2^30");
    if (o->int8_max_k < 0 || o->int8_max_k > 128) return fail(SNP_ERR_INVALID, "int8_max_k must be in 0..128");
    return SNP_OK;
}

// The visited set holds 2^k >= 2 (max_rows + 2 chunk) entries indexed by 32-bit
// slots: max_rows + 2 chunk must not pass 2^31.
snp_status validate_table_size(long long max_rows, long long chunk) {
    if (max_rows + 2 * chunk > (1LL << 31))
        return fail(SNP_ERR_INVALID, "max_rows + 2 * chunk = %lld exceeds 2^31 (visited-set slots are 32-bit)",
                    max_rows + 2 * chunk);
    return SNP_OK;
}

// Wait for a stream by polling it: a pass's counters are awaited many times
// per walk, each a few tens of microseconds after the launch, and a blocking
// wait adds the wake-up of a sleeping thread to every one of them.
hipError_t wait_stream(hipStream_t st) {
    hipError_t e;
    while ((e = hipStreamQuery(st)) == hipErrorNotReady) {
    }
    return e;
}

// Copy the current pass's counters to the host and wait for the stream.  The
// checks of a walk start still unread (in the same slot) are reported first.
snp_status read_counters(snp_system* S) {
    HIPCHK(hipMemcpyAsync(S->h_ctr, S->d_ctr, sizeof(snp::DevCounters), hipMemcpyDeviceToHost, S->stream));
    HIPCHK(wait_stream(S->stream));
    if (S->start_pending) {
        S->start_pending = false;
        if (S->h_ctr->c0_bad) return fail(SNP_ERR_OVERFLOW, "C0 holds a count outside the count type's range");
    }
    return SNP_OK;
}

// Start a device pass: move to the next counter slot (zeroing the ring when it
// wraps, i.e. one fill per kRing passes instead of one per pass).
snp_status clear_counters(snp_system* S) {
    if (S->slot_ready) {  // set up by the walk start, which counted nothing else
        S->slot_ready = false;
        return SNP_OK;
    }
    const int slot = (int)(S->pass % snp_system::kRing);
    if (slot == 0)
        HIPCHK(hipMemsetAsync(S->d_ring, 0, sizeof(snp::DevCounters) * snp_system::kRing, S->stream));
    S->d_ctr = S->d_ring + slot;
    ++S->pass;
    return SNP_OK;
}

// Empty the visited set and insert rows [0, rows) of the row store, counting
// in ctr.
snp_status fill_table(snp_system* S, const void* arena, long long rows, snp::DevCounters* ctr) {
    HIPCHK(snp::launch_fill_u64(S->d_table, (long long)S->slots, snp::kEmpty, S->stream));
    HIPCHK(snp::launch_rows_insert(S->elem_bytes, S->m, S->d_R, S->d_table, S->slots - 1, arena, 0, rows,
                                   S->opt.hash_mask ? S->opt.hash_mask : ~0ULL, S->d_row_slot, ctr, S->stream));
    S->tombs = 0;
    return SNP_OK;
}

// The same as a device pass of its own (drops the tombstones of a long walk).
snp_status rebuild_table(snp_system* S, const void* arena, long long rows) {
    snp_status st;
    if ((st = clear_counters(S))) return st;
    if ((st = fill_table(S, arena, rows, S->d_ctr))) return st;
    if ((st = read_counters(S))) return st;
    if (S->h_ctr->probe_fail) return fail(SNP_ERR_DEVICE, "visited set: no free slot");
    return SNP_OK;
}

// Record C0 as the only visited configuration, stored at arena row 0 (parent
// and child index -1 in par0 / chi0 when given).  Its range check goes to the
// counter slot that the first pass then uses; with `wait` false the result is
// read (and a bad C0 reported) by that pass's counter read, so the first level
// costs no synchronisation of its own.  The kernels never index memory by a
// count, so a level expanded from a bad C0 stays in bounds before the error.
snp_status start_walk(snp_system* S, const void* c0_dev, void* arena, bool wait, long long* par0 = nullptr,
                      long long* chi0 = nullptr, bool psi_c0 = false) {
    if (!c0_dev) return fail(SNP_ERR_INVALID, "c0 is NULL");
    const char *c = (const char*)c0_dev, *a = (const char*)arena;
    if (c != a && c < a + row_bytes(S) && a < c + row_bytes(S))
        return fail(SNP_ERR_INVALID, "c0 overlaps row 0 of the row store without being it");
    S->slot_ready = false;
    snp_status st;
    if ((st = clear_counters(S))) return st;  // the slot the first pass will use
    HIPCHK(snp::launch_start_walk(S->elem_bytes, S->m, S->d_R, S->d_table, S->slots - 1, c0_dev, arena, S->count_max,
                                  S->opt.hash_mask ? S->opt.hash_mask : ~0ULL, S->d_row_slot, S->d_ctr, par0,
                                  chi0, S->dsys, S->opt.expand_max_count, psi_c0 ? S->d_psi : nullptr, S->d_psif,
                                  S->d_hflag, S->d_off, S->d_T, S->stream));
    S->slot_ready = true;
    S->tombs = 0;
    S->start_pending = true;
    return wait ? read_counters(S) : SNP_OK;
}

// A keys-first pass (stage_rows 0) when the chunk's rows reach this many bytes:
// below it the commit's copy costs less than the key pass and the row check.
constexpr double kKeysFirstBytes = 64.0 * 1024 * 1024;

// Up to this many parents the commit block that fills the cap counts the
// halting parents itself (a few loads per thread).
constexpr long long kCommitHaltMax = 1 << 16;

struct LevelIO {
    const void* frontier;
    long long n;
    void* arena;            // row store
    long long level_base;   // rows recorded before this level
    long long arena_cap;    // rows the row store holds
    long long limit_sem;    // frontier_cap (kInf: none)
    long long limit_cap;    // caller buffer capacity (kInf: none)
    void* row2;             // nullable copy destination
    long long* par_out;
    long long par_out_base;
    long long par_value_base;
    long long* t_out;
    bool c0_psi = false;    // the frontier is C0, whose Psi the walk start computed
};

snp_status rollback_level(snp_system* S, long long first, long long count) {
    HIPCHK(snp::launch_rollback(S->d_row_slot, S->d_table, first, count, S->stream));
    HIPCHK(hipStreamSynchronize(S->stream));
    S->tombs += count;
    return SNP_OK;
}

// Joins a children count split at bit 31 (DevCounters::psif_lo / psif_hi),
// saturated at 2^62.
u64 join_full(u64 lo, u64 hi) {
    if (hi >= (1ULL << 31)) return snp::kPsiSat;
    const u64 v = (hi << 31) + lo;
    return v >= snp::kPsiSat ? snp::kPsiSat : v;
}

u64 sat_add_host(u64 a, u64 b) { return std::min<u64>(snp::kPsiSat, a + b); }

// One BFS level: children of io.frontier, deduplicated, committed in order.
// Only canonical children are computed (a child firing the later of two twin
// rules repeats an earlier child of the same parent, so it is never a first
// occurrence); they are numbered level-wide in child order, and chunks cover
// ranges of that numbering.
snp_status expand_level(snp_system* S, const LevelIO& io, snp_expand_stats* out, long long* count_out) {
    snp_expand_stats stt{};
    *count_out = 0;
    stt.parents = io.n;
    stt.int8_fallback = (S->opt.path == SNP_PATH_INT8 && !S->int8_ready) ? 1 : 0;
    // Form of a pass.  The int8 form computes one reference child per segment
    // (consecutive canonical children of one parent, at most 64) by a pull and
    // the rest on the matrix cores; with few canonical children per parent its
    // segments shrink to single children and every child costs a pull plus the
    // matrix-core overhead.  AUTO compares the two per child, with the
    // segment length taken from the canonical children per parent of the
    // prefix examined so far (of the last level before the first pass); the
    // one-neuron-per-lane form is kept wherever it applies.
    auto choose_int8 = [&](double per_parent) -> bool {
        if (S->opt.path == SNP_PATH_INT8) return S->int8_ready;
        if (S->opt.path != SNP_PATH_AUTO || !S->int8_ready || S->lane_form) return false;
        const double seg = std::max(1.0, std::min(64.0, per_parent));
        return S->pull_work / seg + S->int8_row_work < S->pull_work;
    };
    stt.path_used = choose_int8(64.0) ? SNP_PATH_INT8 : SNP_PATH_SPARSE;
    if (io.n > S->max_frontier)
        return fail(SNP_ERR_CAPACITY, "frontier of %lld rows exceeds max_frontier %lld", io.n, S->max_frontier);
    snp_status st;
    if (io.n <= 0) {
        if (out) *out = stt;
        return SNP_OK;
    }
    const u64 hmask = S->opt.hash_mask ? S->opt.hash_mask : ~0ULL;
    const long long rb = row_bytes(S);

    // Psi and child offsets are computed for a growing prefix [0, P) of the
    // frontier, only as far as the chunks need children: a level stopped by
    // its cap usually reaches a small fraction of its parents.  An extension of
    // the prefix runs in the same device pass as the chunk that needs it; the
    // chunk kernels read the prefix's canonical child count on the device and
    // stop there, so a pass costs one host synchronisation.
    long long P = 0;
    u64 T = 0;                  // canonical children of parents [0, P) (saturated), known after each pass
    u64 Tf = 0;                 // all children of parents [0, P) (saturated)
    u64 Tend = 0;               // canonical children the chunks may take: T, or the budget's clip
    long long halting_all = 0;  // halting parents in [0, P)
    const bool has_budget = S->opt.child_budget > 0;
    const u64 budget = has_budget ? (u64)S->opt.child_budget : ~0ULL;
    long long bud_par = 0;      // parent of the budget's last child, + 1
    u64* d_end = has_budget ? S->d_Tend : S->d_T;
    // The first extension of a level covers 4096 parents, or fewer (not under
    // 1024) when the last level's children per parent say that enough for the
    // first chunk lie in fewer; later ones double the prefix.
    auto launch_extension = [&](u64 want) -> snp_status {
        long long grow = std::max<long long>(4096, P);
        if (P == 0 && want > 0 && S->psi_per_parent > 0.0) {
            const double need = (double)want / S->psi_per_parent * 1.5 + 64.0;
            grow = std::min<long long>(grow, std::max<long long>(1024, (long long)need));
        }
        const long long P1 = std::min(io.n, P + grow);
        const char* f = (const char*)io.frontier + P * rb;
        if (snp::psi_scan_fits(S->dsys, P1 - P)) {  // a few small parents: one launch
            HIPCHK(snp::launch_psi_scan_small(S->elem_bytes, S->dsys, f, P1 - P, S->opt.expand_max_count,
                                              S->d_psi + P, S->d_psif + P, S->d_hflag + P, S->d_off + P,
                                              P == 0 ? nullptr : S->d_T, S->d_T, S->d_ctr, S->stream));
        } else {
            HIPCHK(snp::launch_psi(S->elem_bytes, S->dsys, f, P1 - P, S->opt.expand_max_count, S->d_psi + P,
                                   S->d_psif + P, S->d_hflag + P, S->d_ctr, S->stream));
            HIPCHK(snp::launch_scan_u64(S->d_psi + P, S->d_off + P, P1 - P, S->d_sc_sums, S->d_sc_pre, S->d_T,
                                        P == 0 ? nullptr : S->d_T, &S->d_ctr->psi_total, S->stream));
        }
        if (has_budget)
            HIPCHK(snp::launch_budget_clip(S->elem_bytes, S->dsys, io.frontier, P1, S->d_psif, S->d_off, S->d_T,
                                           budget, S->d_Tend, S->d_ctr, S->stream));
        P = P1;
        return SNP_OK;
    };
    // after an extension pass: the prefix's totals
    auto take_extension = [&](const snp::DevCounters& c) {
        T = c.psi_total;
        Tf = sat_add_host(Tf, join_full(c.psif_lo, c.psif_hi));
        halting_all += (long long)c.halting;
        Tend = has_budget ? c.tend : T;
        if (has_budget && c.bud_par) bud_par = (long long)c.bud_par;
    };

    const long long cap_limit = std::min(io.limit_cap, io.arena_cap - io.level_base);
    const long long limit = std::min(io.limit_sem, cap_limit);
    const bool sem_binds = io.limit_sem <= cap_limit;
    long long count = 0;
    u64 G = 0;                 // canonical children taken by the chunks so far
    u64 enumerated = 0;        // children (all, in child order) up to where the level stopped
    u64 canon_enumerated = 0;  // canonical ones among them
    bool cap_hit = false, budget_hit = false;
    // C0's Psi, halting flag and offset come from the walk start, into the
    // counters of this level's first pass: that pass extends by nothing
    bool start_ext = io.c0_psi && S->slot_ready;
    if (start_ext) P = 1;
    long long halting_cap = -1;  // halting parents up to the cap's child's parent, counted in its pass
    bool redo_staged = false;    // the last pass was keys-first and failed its row check
    for (;;) {
        u64 want = (u64)S->chunk_eff;
        if (io.limit_sem < kInf) {
            const double ratio = std::max(S->new_ratio, 1.0 / 64.0);
            const double w = (double)(io.limit_sem - count) / ratio * 1.1 + 1024.0;
            if (w < (double)want) want = (u64)std::max<double>(w, 4096.0);
        }
        // the prefix needs no extension once it holds the budget's last child
        const bool can_extend = P < io.n && !(has_budget && Tf >= budget);
        const bool ext = start_ext || (can_extend && Tend - G < want);
        if (!ext && Tend <= G) break;  // every child the level may take was enumerated
        const long long B = (long long)(ext ? want : std::min<u64>(want, Tend - G));  // upper bound when extending
        // keep the table at most half full (tombstones included)
        const long long live = io.level_base + count;
        if ((u64)(live + S->tombs + B) * 2 > S->slots) {
            if (start_ext) {  // the rebuild takes the start's counters: compute C0's Psi in the pass
                start_ext = false;
                P = 0;
            }
            if ((st = rebuild_table(S, io.arena, live))) return st;
            if ((u64)(live + B) * 2 > S->slots)
                return fail(SNP_ERR_CAPACITY, "visited set too small for %lld rows", live + B);
        }
        // canonical children per parent: of the prefix examined by the earlier
        // passes of the level, else of the last level (64 before any)
        const double per_parent = G > 0 && P > 0 && T > 0 ? (double)T / (double)P
                                  : (S->psi_per_parent > 0.0 ? S->psi_per_parent : 64.0);
        if ((st = clear_counters(S))) return st;
        if ((st = mark(S, 0))) return st;
        if (ext && !start_ext && (st = launch_extension(want))) return st;
        const bool ext_c0 = start_ext;
        start_ext = false;
        if ((st = mark(S, 1))) return st;
        snp::ChunkArgs ca{io.frontier, P, S->d_psi, S->d_off, G, B, S->d_stage, S->d_hash, S->d_cpar, S->d_ct,
                          hmask, S->d_ctr, d_end, S->opt.int8_max_k > 0 ? S->opt.int8_max_k : 128,
                          S->tune_tiles, S->tune_run, S->d_table, S->slots - 1, S->d_slot, S->d_cand};
        if (ext_c0 && has_budget)  // C0's clip, from the Psi the walk start computed
            HIPCHK(snp::launch_budget_clip(S->elem_bytes, S->dsys, io.frontier, 1, S->d_psif, S->d_off, S->d_T,
                                           budget, S->d_Tend, S->d_ctr, S->stream));
        bool probed = false;
        const bool use_int8 = choose_int8(per_parent);
        stt.path_used = use_int8 ? SNP_PATH_INT8 : SNP_PATH_SPARSE;
        // keys-first: keys, probe and flags, then every row once (new rows
        // straight to the row store), then the row check
        const bool direct = use_int8 && !redo_staged && io.row2 == nullptr && S->opt.stage_rows <= 0 &&
                            (S->opt.stage_rows < 0 || (double)B * (double)rb >= kKeysFirstBytes);
        snp::TableArgs ta{S->d_table, S->slots - 1, io.arena, S->d_stage, S->d_hash, S->d_slot, B, S->d_ctr,
                          S->d_cand, direct ? 1 : 0};
        if (direct) {
            ca.mode = 1;  // keys, each probed in the visited set by the kernel itself
            HIPCHK(snp::launch_expand_int8(S->elem_bytes, S->dsys, ca, S->stream));
            HIPCHK(snp::launch_flags(S->d_table, S->d_slot, B, S->d_ctr, S->d_flag, S->d_pos, S->d_fsums,
                                     S->d_fpre, S->stream, true));
            if ((st = mark(S, 1))) return st;
            ca.mode = 2;
            ca.flag = S->d_flag;
            ca.pos = S->d_pos;
            ca.tile_pre = S->d_fpre;
            ca.arena = io.arena;
            ca.arena_row = io.level_base + count;
            ca.limit_new = limit - count;
            HIPCHK(snp::launch_expand_int8(S->elem_bytes, S->dsys, ca, S->stream));
            if ((st = mark(S, 2))) return st;
            const snp::VerifyArgs va{S->d_table, S->d_slot, S->d_stage, io.arena, S->d_flag, S->d_pos, S->d_fpre,
                                     io.level_base + count, limit - count, B, S->d_ctr};
            HIPCHK(snp::launch_verify(S->elem_bytes, S->m, va, S->stream));
            if ((st = mark(S, 3))) return st;
        } else {
            if (use_int8) HIPCHK(snp::launch_expand_int8(S->elem_bytes, S->dsys, ca, S->stream));
            else HIPCHK(snp::launch_expand_sparse(S->elem_bytes, S->dsys, ca, S->stream, &probed));
            if ((st = mark(S, 2))) return st;
            HIPCHK(snp::launch_insert(S->elem_bytes, S->m, ta, S->stream, !probed));
            if ((st = mark(S, 3))) return st;
            HIPCHK(snp::launch_flags(S->d_table, S->d_slot, B, S->d_ctr, S->d_flag, S->d_pos, S->d_fsums,
                                     S->d_fpre, S->stream));
        }
        if ((st = mark(S, 4))) return st;
        snp::CommitArgs cm{S->d_table, S->d_table, S->d_slot, S->d_hash, S->d_pos, S->d_flag, S->d_fsums, S->d_fpre,
                           S->d_stage, S->d_cpar, S->d_ct, S->d_psif, B, io.arena, io.level_base, count, limit,
                           io.row2, io.par_out, io.par_out_base, io.par_value_base, io.t_out, S->d_row_slot,
                           S->d_ctr, nullptr, direct ? 0 : 1};
        // when this pass may fill the cap, count the halting parents (and the
        // children of the parents) up to the parent of the cap's child in the
        // same pass (no extra synchronisation): in the commit block that fills
        // it, or for many parents in a kernel of its own
        const bool may_cap = sem_binds && B >= limit - count;
        if (may_cap && P <= kCommitHaltMax) cm.hflag = S->d_hflag;
        HIPCHK(snp::launch_commit(S->elem_bytes, S->m, cm, S->stream));
        if (may_cap && P > kCommitHaltMax)
            HIPCHK(snp::launch_count_flags_cap(S->d_hflag, S->d_psif, P, S->d_ctr, S->stream));
        if ((st = mark(S, 5))) return st;
        if ((st = read_counters(S))) return st;
        if (S->opt.profile == 1) {
            if ((st = add_elapsed(S, 1, 2, &stt.ns_expand))) return st;
        } else if (S->opt.profile >= 2) {
            if ((st = add_elapsed(S, 0, 1, &stt.ns_psi))) return st;
            if ((st = add_elapsed(S, 1, 2, &stt.ns_expand))) return st;
            if ((st = add_elapsed(S, 2, 3, &stt.ns_insert))) return st;
            if ((st = add_elapsed(S, 3, 4, &stt.ns_flags))) return st;
            if ((st = add_elapsed(S, 4, 5, &stt.ns_commit))) return st;
        }
        const snp::DevCounters c = *S->h_ctr;
        if (c.probe_fail) return fail(SNP_ERR_DEVICE, "visited set: probe found no free slot");
        if (direct && c.verify_fail) {
            // a key named a configuration whose row differs: undo the pass
            // (the entries of the rows it recorded become tombstones, like those
            // of new children past the limit) and redo it with staged rows
            const long long new_total = (long long)c.total;
            const long long committed = std::min(new_total, limit - count);
            S->tombs += new_total - committed;
            if (committed > 0 && (st = rollback_level(S, io.level_base + count, committed))) return st;
            if (ext) take_extension(c);
            ++stt.redone;
            redo_staged = true;
            continue;
        }
        redo_staged = false;
        if (direct) ++stt.keys_first;
        if (ext) take_extension(c);
        const long long Beff = (long long)c.beff;
        if (Beff > 0) ++stt.chunks;
        if (Beff > 0 && stt.path_used == SNP_PATH_INT8) ++stt.int8_chunks;
        stt.expanded += Beff;
        stt.collisions += (long long)c.collisions;
        stt.mfma_ops += (long long)c.mfma * 32768;
        const long long new_total = (long long)c.total;
        const long long avail = limit - count;
        const long long committed = std::min(new_total, avail);
        S->tombs += new_total - committed;  // new children past the limit became tombstones
        if (c.overflow) {
            if ((st = rollback_level(S, io.level_base, count + committed))) return st;
            *count_out = count;
            return fail(SNP_ERR_OVERFLOW, "a child configuration holds a count above %lld", S->count_max);
        }
        if (Beff > 0) S->new_ratio = (double)new_total / (double)Beff;
        if (new_total >= avail && sem_binds && avail > 0) {
            count = limit;
            cap_hit = true;
            // the cap child: canonical index G + cap_g - 1; index among all
            // children = all children of the parents before its parent + its t
            canon_enumerated = G + c.cap_g;
            enumerated = sat_add_host(sat_add_host(join_full(c.capf_lo, c.capf_hi), c.cap_t), 1);
            halting_cap = (long long)c.count;
            break;
        }
        if (new_total > avail) {
            if ((st = rollback_level(S, io.level_base, count + committed))) return st;
            *count_out = count + new_total;
            return fail(SNP_ERR_CAPACITY, "level needs more than %lld rows", cap_limit);
        }
        count += new_total;
        G += (u64)Beff;
    }
    if (!cap_hit) {
        canon_enumerated = G;
        if (has_budget && Tf >= budget) {
            // the budget's last child was reached: is any child left after it?
            while (Tf <= budget && P < io.n) {
                if ((st = clear_counters(S))) return st;
                if ((st = launch_extension(0))) return st;
                if ((st = read_counters(S))) return st;
                take_extension(*S->h_ctr);
            }
            budget_hit = Tf > budget;
        }
        enumerated = budget_hit ? budget : Tf;
    }
    // halting parents up to the parent of the last enumerated child (all parents
    // when the level was not cut short by the cap or the budget)
    if (cap_hit) {
        stt.halting_parents = halting_cap;
    } else if (budget_hit) {
        if ((st = clear_counters(S))) return st;
        HIPCHK(snp::launch_count_flags(S->d_hflag, bud_par, &S->d_ctr->count, S->stream));
        if ((st = read_counters(S))) return st;
        stt.halting_parents = (long long)S->h_ctr->count;
    } else {
        stt.halting_parents = halting_all;
    }
    if (P > 0) S->psi_per_parent = (double)T / (double)P;
    stt.children_total = (long long)Tf;
    stt.enumerated = (long long)enumerated;
    stt.twins = (long long)(enumerated - std::min(enumerated, canon_enumerated));
    stt.new_configs = count;
    stt.duplicates = (long long)enumerated - count;
    stt.truncated = cap_hit ? 1 : 0;
    stt.budget_hit = budget_hit ? 1 : 0;
    if (out) *out = stt;
    *count_out = count;
    return SNP_OK;
}

}  // namespace

extern "C" {

const char* snp_last_error(void) { return g_err.c_str(); }

int64_t snp_row_bytes(const snp_system* S) { return S ? row_bytes(S) : 0; }

void snp_free(snp_system* S) { delete S; }

snp_status snp_load(const snp_desc* d, const snp_options* o, snp_system** out) {
    g_err.clear();
    if (!out) return fail(SNP_ERR_INVALID, "out is NULL");
    *out = nullptr;
    snp_status st = validate(d);
    if (st) return st;
    snp_options opt{};
    if (o) opt = *o;
    else opt.max_rows = 1 << 20;
    if ((st = validate_options(&opt))) return st;

    // Definition 2 cross-check of a caller-supplied M, and the int8 range test.
    std::vector<std::vector<char>> adj(d->m, std::vector<char>(d->m, 0));
    for (int e = 0; e < d->n_syn; ++e) adj[d->syn_src[e]][d->syn_dst[e]] = 1;
    bool int8_ok = true;
    for (int k = 0; k < d->r; ++k) {
        if (d->rule_c[k] > 127 || d->rule_p[k] > 127) int8_ok = false;
        if (d->M)
            for (int n = 0; n < d->m; ++n) {
                const int want = def2_entry(d, adj, k, n);
                if (d->M[(long long)k * d->m + n] != want)
                    return fail(SNP_ERR_INVALID, "M[%d][%d] = %d but Definition 2 gives %d", k, n,
                                d->M[(long long)k * d->m + n], want);
            }
    }

    // An output neuron adds two entries to every row (its spike train), and
    // with delays every neuron owning a rule with a delay adds two more (its
    // wait and pending spikes), all read and written by the kernels: the
    // device tables see that many more neurons, without rules or synapses.
    if (opt.out_neuron < 0 || opt.out_neuron > d->m)
        return fail(SNP_ERR_INVALID, "out_neuron %d outside [0, m = %d]", opt.out_neuron, d->m);
    const int mcount = d->m;
    const int dfirst = mcount + (opt.out_neuron > 0 ? 2 : 0);
    std::vector<int> dlink;  // neuron -> its wait column (-1: none); state column -> its neuron
    int width = dfirst;
    if (d->rule_d) {
        std::vector<char> delayed(mcount, 0);
        for (int k = 0; k < d->r; ++k)
            if (d->rule_d[k] > 0) delayed[d->rule_neuron[k]] = 1;
        dlink.assign(mcount, -1);
        for (int n = 0; n < mcount; ++n)
            if (delayed[n]) {
                dlink[n] = width;
                width += 2;
            }
        if (width == dfirst) dlink.clear();  // every delay 0: the system without delays
        else {
            dlink.resize(width, -1);
            for (int n = 0; n < mcount; ++n)
                if (dlink[n] >= 0) dlink[dlink[n]] = dlink[dlink[n] + 1] = n;
        }
    }
    const bool delays = !dlink.empty();
    if (width > (delays ? kMaxDelayWidth : kMaxNeurons))
        return fail(SNP_ERR_INVALID, "row width %d (counts, output spike train, delay states) above %d", width,
                    delays ? kMaxDelayWidth : kMaxNeurons);
    snp_desc wide;
    if (width > mcount) {
        wide = *d;
        wide.m = width;
        wide.M = nullptr;
        d = &wide;
    }

    snp_system* S = new snp_system();
    S->m = d->m;
    S->r = d->r;
    S->mcount = mcount;
    S->delays = delays;
    S->track = opt.out_neuron > 0 ? mcount : -1;
    S->elem_bytes = d->count_type == SNP_COUNT_U16 ? 2 : 4;
    S->count_max = d->count_type == SNP_COUNT_U16 ? 65535 : INT_MAX;
    S->opt = opt;
    S->stream = (hipStream_t)opt.stream;
    S->int8_ok = int8_ok;
    S->max_rows = opt.max_rows;
    S->max_frontier = opt.max_frontier > 0 ? opt.max_frontier : opt.max_rows;
    const long long rb = row_bytes(S);
    S->chunk_max = opt.chunk > 0 ? opt.chunk : std::min<long long>(1 << 20, std::max<long long>(4096, (1LL << 28) / rb));
    S->chunk_eff = S->chunk_max;
    if ((st = validate_table_size(S->max_rows, S->chunk_max))) {
        delete S;
        return st;
    }
    static std::atomic<unsigned long long> next_uid{1};
    S->uid = next_uid++;
    S->count_type = d->count_type;
    S->h_rn.assign(d->rule_neuron, d->rule_neuron + d->r);
    S->h_ri.assign(d->rule_i, d->rule_i + d->r);
    S->h_rj.assign(d->rule_j, d->rule_j + d->r);
    S->h_rc.assign(d->rule_c, d->rule_c + d->r);
    S->h_rp.assign(d->rule_p, d->rule_p + d->r);
    S->h_ss.assign(d->syn_src, d->syn_src + d->n_syn);
    S->h_sd.assign(d->syn_dst, d->syn_dst + d->n_syn);

    // rule tables (rules of a neuron are contiguous: validated order)
    std::vector<int> nrule_ptr(d->m + 1, 0);
    for (int k = 0; k < d->r; ++k) nrule_ptr[d->rule_neuron[k] + 1]++;
    for (int n = 0; n < d->m; ++n) nrule_ptr[n + 1] += nrule_ptr[n];
    std::vector<int4> rules(d->r);
    // (with delays the last entry packs p and the delay d: p | d << 16)
    for (int k = 0; k < d->r; ++k)
        rules[k] = make_int4(d->rule_i[k], d->rule_j[k], d->rule_c[k],
                             d->rule_p[k] | (delays ? d->rule_d[k] << 16 : 0));
    // in-synapses of every neuron (column view of the synapse part of M)
    // (one padding entry, so kernels may read in_src[0] of a system without synapses)
    std::vector<int> in_ptr(d->m + 1, 0), in_src(std::max(1, d->n_syn), 0), fill(d->m, 0);
    for (int e = 0; e < d->n_syn; ++e) in_ptr[d->syn_dst[e] + 1]++;
    for (int n = 0; n < d->m; ++n) in_ptr[n + 1] += in_ptr[n];
    for (int e = 0; e < d->n_syn; ++e) {
        const int t = d->syn_dst[e];
        in_src[in_ptr[t] + fill[t]++] = d->syn_src[e];
    }
    for (int n = 0; n < d->m; ++n) std::sort(in_src.begin() + in_ptr[n], in_src.begin() + in_ptr[n + 1]);

    auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
        if (bytes == 0) return hipSuccess;
        return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    };
#define LOADCHK(expr)                                                                                \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) {                                                                      \
            delete S;                                                                                \
            return fail(SNP_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));                    \
        }                                                                                            \
    } while (0)
    LOADCHK(dmalloc(&S->d_nrule_ptr, sizeof(int) * (d->m + 1)));
    LOADCHK(dmalloc(&S->d_rules, sizeof(int4) * d->r));
    LOADCHK(dmalloc(&S->d_in_ptr, sizeof(int) * (d->m + 1)));
    LOADCHK(dmalloc(&S->d_in_src, sizeof(int) * in_src.size()));
    LOADCHK(up(S->d_nrule_ptr, nrule_ptr.data(), sizeof(int) * (d->m + 1)));
    LOADCHK(up(S->d_rules, rules.data(), sizeof(int4) * d->r));
    LOADCHK(up(S->d_in_ptr, in_ptr.data(), sizeof(int) * (d->m + 1)));
    LOADCHK(up(S->d_in_src, in_src.data(), sizeof(int) * in_src.size()));
    if (delays) {
        LOADCHK(dmalloc(&S->d_dlink, sizeof(int) * dlink.size()));
        LOADCHK(up(S->d_dlink, dlink.data(), sizeof(int) * dlink.size()));
    }
    // hash weights R[n] and the hash H of every row of M_Pi (Definition 2 rows,
    // entries sign-extended, arithmetic mod 2^64)
    std::vector<u64> R(d->m), hM(d->r);
    for (int n = 0; n < d->m; ++n) R[n] = host_mix64((u64)(n + 1) * 0x9E3779B97F4A7C15ULL);
    std::vector<std::vector<int>> outs(d->m);
    for (int e = 0; e < d->n_syn; ++e) outs[d->syn_src[e]].push_back(d->syn_dst[e]);
    int max_rules = 0;
    for (int n = 0; n < d->m; ++n) max_rules = std::max(max_rules, nrule_ptr[n + 1] - nrule_ptr[n]);
    for (int k = 0; k < d->r; ++k) {
        const int src = d->rule_neuron[k];
        u64 h = (u64)(-(long long)d->rule_c[k]) * R[src];
        for (int t : outs[src]) h += (u64)(long long)d->rule_p[k] * R[t];
        hM[k] = h;
    }
    LOADCHK(dmalloc(&S->d_R, sizeof(u64) * d->m));
    LOADCHK(dmalloc(&S->d_hM, sizeof(u64) * d->r));
    LOADCHK(up(S->d_R, R.data(), sizeof(u64) * d->m));
    LOADCHK(up(S->d_hM, hM.data(), sizeof(u64) * d->r));
    // int8 copy of M_Pi for the matrix-core form (every |entry| <= 127, <= 16 rules per neuron)
    S->int8_ready = int8_ok && S->track < 0 && !delays && max_rules <= 16 && opt.path != SNP_PATH_SPARSE &&
                    snp::int8_lds(d->m, 64) <= 64 * 1024 && (size_t)d->r * d->m <= ((size_t)1 << 33);
    if (S->int8_ready) {
        std::vector<int8_t> M8((size_t)d->r * d->m, 0);
        for (int k = 0; k < d->r; ++k) {
            const int src = d->rule_neuron[k];
            M8[(size_t)k * d->m + src] = (int8_t)(-d->rule_c[k]);
            for (int t : outs[src]) M8[(size_t)k * d->m + t] = (int8_t)d->rule_p[k];
        }
        LOADCHK(dmalloc(&S->d_M8, M8.size()));
        LOADCHK(up(S->d_M8, M8.data(), M8.size()));
    }
    // per-child work of the two forms: the pull visits every neuron and synapse;
    // the matrix-core form adds the row's matrix-core product and store
    S->pull_work = (double)d->m + (double)d->n_syn;
    S->int8_row_work = (double)d->m * 1.5;
    int max_in = 0;
    for (int n = 0; n < d->m; ++n) max_in = std::max(max_in, in_ptr[n + 1] - in_ptr[n]);
    // lane-major in-synapse table of the one-neuron-per-lane expansion
    std::vector<int> in_lane(16 * 64, -1);
    if (d->m <= 64 && max_in <= 16)
        for (int n = 0; n < d->m; ++n)
            for (int e = 0; e < in_ptr[n + 1] - in_ptr[n]; ++e) in_lane[e * 64 + n] = in_src[in_ptr[n] + e];
    LOADCHK(dmalloc(&S->d_in_lane, sizeof(int) * in_lane.size()));
    LOADCHK(up(S->d_in_lane, in_lane.data(), sizeof(int) * in_lane.size()));
    S->lane_form = S->track < 0 && !delays && d->m <= 64 && max_in <= 16 && (size_t)d->r * 24 <= 24 * 1024;
    S->dsys = snp::DevSystem{d->m, d->r, S->d_nrule_ptr, S->d_rules, S->d_in_ptr, S->d_in_src, d->n_syn, S->d_M8,
                             S->count_max, S->d_R, S->d_hM, max_in, S->d_in_lane,
                             opt.deterministic ? 1ULL : snp::kPsiSat, S->track,
                             opt.out_neuron > 0 ? opt.out_neuron - 1 : -1, S->d_dlink, mcount, dfirst};

    S->slots = next_pow2((u64)std::max<long long>(1024, 2 * (S->max_rows + 2 * S->chunk_max)));
    LOADCHK(dmalloc(&S->d_table, sizeof(u64) * S->slots));
    LOADCHK(dmalloc(&S->d_row_slot, sizeof(uint32_t) * S->max_rows));
    const long long F = S->max_frontier;
    LOADCHK(dmalloc(&S->d_psi, sizeof(u64) * F));
    LOADCHK(dmalloc(&S->d_psif, sizeof(u64) * F));
    LOADCHK(dmalloc(&S->d_hflag, (size_t)F));
    LOADCHK(dmalloc(&S->d_off, sizeof(u64) * F));
    const long long ft = snp::scan_tiles(std::max(F, S->chunk_max)) + 1;
    LOADCHK(dmalloc(&S->d_sc_sums, sizeof(u64) * ft));
    LOADCHK(dmalloc(&S->d_sc_pre, sizeof(u64) * ft));
    const long long C = S->chunk_max;
    LOADCHK(dmalloc(&S->d_stage, (size_t)(C * rb)));
    LOADCHK(dmalloc(&S->d_hash, sizeof(u64) * C));
    LOADCHK(dmalloc(&S->d_cpar, sizeof(int) * C));
    LOADCHK(dmalloc(&S->d_ct, sizeof(u64) * C));
    LOADCHK(dmalloc(&S->d_slot, sizeof(uint32_t) * C));
    LOADCHK(dmalloc(&S->d_cand, sizeof(uint32_t) * C));
    LOADCHK(dmalloc(&S->d_flag, sizeof(uint32_t) * C));
    LOADCHK(dmalloc(&S->d_pos, sizeof(uint32_t) * C));
    LOADCHK(dmalloc(&S->d_fsums, sizeof(uint32_t) * ft));
    LOADCHK(dmalloc(&S->d_fpre, sizeof(uint32_t) * ft));
    LOADCHK(dmalloc(&S->d_ring, sizeof(snp::DevCounters) * snp_system::kRing));
    LOADCHK(dmalloc(&S->d_T, sizeof(u64)));
    LOADCHK(dmalloc(&S->d_Tend, sizeof(u64)));
    S->d_ctr = S->d_ring;
    LOADCHK(hipHostMalloc((void**)&S->h_ctr, sizeof(snp::DevCounters), hipHostMallocDefault));
    if (opt.profile)
        // timing only: no system-scope fence when an event is reached
        for (hipEvent_t& e : S->ev) LOADCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
#undef LOADCHK
    *out = S;
    return SNP_OK;
}

snp_status snp_reset(snp_system* S, const void* c0_dev) {
    g_err.clear();
    if (!S) return fail(SNP_ERR_INVALID, "handle is NULL");
    if (!S->d_store) HIPCHK(dmalloc(&S->d_store, (size_t)(S->max_rows * row_bytes(S))));
    S->walk_active = false;
    snp_status st = start_walk(S, c0_dev, S->d_store, true);
    if (st) return st;
    S->walk_active = true;
    S->walk_rows = 1;
    return SNP_OK;
}

snp_status snp_expand(snp_system* S, const void* frontier_dev, int64_t n, void* next_dev, int64_t next_capacity,
                      int64_t* n_next, int64_t* parent_of_next, int64_t* child_of_next, snp_expand_stats* stats) {
    g_err.clear();
    if (!S) return fail(SNP_ERR_INVALID, "handle is NULL");
    if (!n_next) return fail(SNP_ERR_INVALID, "n_next is NULL");
    *n_next = 0;
    if (!S->walk_active) return fail(SNP_ERR_INVALID, "snp_expand before snp_reset");
    if (n < 0 || next_capacity < 0) return fail(SNP_ERR_INVALID, "negative n or next_capacity");
    if (n > 0 && !frontier_dev) return fail(SNP_ERR_INVALID, "frontier is NULL");
    if (next_capacity > 0 && !next_dev) return fail(SNP_ERR_INVALID, "next is NULL");
    const long long rb = row_bytes(S);
    const char* f0 = (const char*)frontier_dev;
    const char* n0 = (const char*)next_dev;
    if (n > 0 && next_capacity > 0 && f0 < n0 + next_capacity * rb && n0 < f0 + n * rb)
        return fail(SNP_ERR_INVALID, "frontier and next buffers overlap");
    LevelIO io{frontier_dev, n, S->d_store, S->walk_rows, S->max_rows,
               S->opt.frontier_cap > 0 ? S->opt.frontier_cap : kInf, next_capacity, next_dev,
               (long long*)parent_of_next, 0, 0, (long long*)child_of_next};
    long long count = 0;
    snp_status st = expand_level(S, io, stats, &count);
    *n_next = count;
    if (st) return st;
    S->walk_rows += count;
    return SNP_OK;
}

snp_status snp_run(snp_system* S, const void* c0_dev, int32_t max_depth, void* out_dev, int64_t out_capacity,
                   int64_t* n_configs, int64_t* level_sizes, int32_t max_levels, int32_t* n_levels,
                   int32_t* stop_reason, snp_expand_stats* level_stats, int64_t* parent_of,
                   int64_t* child_of) {
    g_err.clear();
    if (!S) return fail(SNP_ERR_INVALID, "handle is NULL");
    if (!out_dev || !n_configs || !level_sizes || !n_levels || !stop_reason)
        return fail(SNP_ERR_INVALID, "out, n_configs, level_sizes, n_levels and stop_reason are required");
    if (out_capacity < 1 || max_levels < 1) return fail(SNP_ERR_CAPACITY, "out_capacity and max_levels must be >= 1");
    *n_configs = 0;
    *n_levels = 0;
    *stop_reason = SNP_STOP_DEPTH;
    S->walk_active = false;
    const long long rb = row_bytes(S);
    snp_status st = start_walk(S, c0_dev, out_dev, false, (long long*)parent_of, (long long*)child_of, true);
    if (st) return st;
    // level_stats entries [0, *n_levels): each expansion writes its own, the
    // rest (levels that were not expanded) are zeroed on the way out
    int32_t written = 0;
    auto done = [&](snp_status r) -> snp_status {
        if (level_stats)
            for (int32_t k = written; k < std::min(*n_levels, max_levels); ++k) level_stats[k] = snp_expand_stats{};
        return r;
    };
    const long long arena_cap = std::min<long long>(out_capacity, S->max_rows);
    long long rows = 1, lv_begin = 0, lv_end = 1;
    int32_t levels = 1;
    level_sizes[0] = 1;
    *n_configs = 1;
    *n_levels = 1;
    int32_t stop = SNP_STOP_DEPTH;
    for (;;) {
        const int32_t depth = levels - 1;
        if (max_depth >= 0 && depth >= max_depth) {
            stop = SNP_STOP_DEPTH;
            break;
        }
        if (levels >= max_levels) {
            HIPCHK(hipStreamSynchronize(S->stream));
            return done(fail(SNP_ERR_CAPACITY, "more than max_levels = %d levels", max_levels));
        }
        LevelIO io{(const char*)out_dev + lv_begin * rb, lv_end - lv_begin, out_dev, rows, arena_cap,
                   S->opt.frontier_cap > 0 ? S->opt.frontier_cap : kInf, kInf, nullptr, (long long*)parent_of,
                   rows, lv_begin, (long long*)child_of, depth == 0};
        snp_expand_stats es{};
        long long count = 0;
        st = expand_level(S, io, &es, &count);
        if (st) {
            if (st == SNP_ERR_CAPACITY && rows + count > arena_cap)
                st = fail(SNP_ERR_CAPACITY, "run needs more than %lld rows (out_capacity or max_rows)", arena_cap);
            return done(st);
        }
        if (level_stats) level_stats[depth] = es;
        written = depth + 1;
        const bool all_halting = es.halting_parents == es.parents;
        if (count > 0) {
            level_sizes[levels++] = count;
            lv_begin = lv_end;
            lv_end = rows + count;
            rows += count;
            *n_configs = rows;
            *n_levels = levels;
        }
        if (all_halting) { stop = SNP_STOP_ALL_HALTING; break; }
        if (es.truncated && S->opt.stop_at_cap) { stop = SNP_STOP_CAP; break; }
        if (es.budget_hit) { stop = SNP_STOP_BUDGET; break; }
        if (count == 0) { stop = SNP_STOP_EMPTY_FRONTIER; break; }
    }
    *stop_reason = stop;
    if (S->start_pending) return done(read_counters(S));  // no level ran: check C0 now
    HIPCHK(hipStreamSynchronize(S->stream));
    return done(SNP_OK);
}

// Checkpoint rows per system of a deterministic run of `steps` steps (one
// every batch_interval() steps, step 0 included), and slots per system of its
// H set (at most half full).
static long long batch_ckpt_rows(int steps) { return steps / snp::batch_interval() + 1; }
static u64 batch_table_slots(int steps) { return next_pow2((u64)std::max(64, 2 * (steps + 1))); }

// Multiplier m of the exact quotient x / d for every 32-bit x and 2 <= d < 2^8
// (Granlund and Montgomery, 1994): with l = ceil(log2 d) and t = mulhi(m, x),
// x / d = (t + ((x - t) >> 1)) >> (l - 1).  0 for d < 2 (not used).
static uint32_t div_magic(uint32_t d) {
    if (d < 2) return 0;
    uint32_t l = 0;
    while ((1u << l) < d) ++l;
    return (uint32_t)(((1ULL << 32) * ((1ULL << l) - d)) / d + 1);
}

// Where the batched kernel reads each in-synapse source.  A wave pulls the
// production words of its 64 slots' sources in P rounds (the wave's largest
// in-degree, capped at 32, rounded up to a multiple of 4), one LDS read per round; LDS
// serves a half-wave (32 lanes) per cycle from 32 four-byte banks, and a
// bank holding several addresses in one round serialises them (one address
// read by many lanes is a broadcast).  Word s of a production buffer is in
// bank s mod 32; 32 zero words, one per bank, follow the slots.  For each
// half-wave and round, in round order: the lanes with the fewest spare
// rounds choose first; a lane takes the source of its own (up to 32) whose
// bank is least loaded in the round, or, when that bank is taken and it has a
// round to spare, nothing; lanes with nothing read a zero word in a free bank.
// reg receives kRegSrc entries per slot: a source slot, or kZeroWord | bank.
// The sources past the first kRegSrc of a slot stay at the end of its list.
static constexpr int kRegSrc = 32;
static constexpr uint16_t kZeroWord = 0xFFE0;
static bool place_in_synapses(int m, const std::vector<int>& ptr, const std::vector<int>& src,
                              std::vector<uint16_t>& reg) {
    reg.assign((size_t)m * kRegSrc, 0);
    for (int g = 0; g < m; g += 64) {
        const int g1 = std::min(m, g + 64);
        int kw = 0;
        for (int j = g; j < g1; ++j) kw = std::max(kw, std::min(kRegSrc, ptr[j + 1] - ptr[j]));
        const int P = std::max(4, (kw + 3) & ~3);
        for (int h = g; h < g1; h += 32) {
            const int h1 = std::min(g1, h + 32);
            std::vector<std::vector<int>> rest(h1 - h);
            for (int j = h; j < h1; ++j)
                rest[j - h].assign(src.begin() + ptr[j], src.begin() + ptr[j] + std::min(kRegSrc, ptr[j + 1] - ptr[j]));
            std::vector<int> order(h1 - h);
            for (int e = 0; e < kRegSrc; ++e) {
                int load[32] = {0}, addr[32];
                for (int b = 0; b < 32; ++b) addr[b] = -1;
                std::vector<int> got(h1 - h, -1);
                if (e < P) {
                    for (int l = 0; l < h1 - h; ++l) order[l] = l;
                    std::stable_sort(order.begin(), order.end(),
                                     [&](int x, int y) { return rest[x].size() > rest[y].size(); });
                    for (int l : order) {
                        std::vector<int>& r = rest[l];
                        if (r.empty()) continue;
                        int best = 0, best_cost = 1 << 30;
                        for (int q = 0; q < (int)r.size(); ++q) {
                            const int b = r[q] & 31;
                            const int c = addr[b] == r[q] ? 0 : load[b];
                            if (c < best_cost) best_cost = c, best = q;
                        }
                        const int spare = P - e - (int)r.size();
                        if (best_cost > 0 && spare > 0) continue;
                        const int v = r[best], b = v & 31;
                        if (addr[b] != v) ++load[b], addr[b] = v;
                        got[l] = v;
                        r.erase(r.begin() + best);
                    }
                }
                // zero words: free banks first, then one already read (a broadcast)
                int zb = -1;
                for (int l = 0; l < h1 - h; ++l) {
                    if (got[l] >= 0) {
                        reg[(size_t)(h + l) * kRegSrc + e] = (uint16_t)got[l];
                        continue;
                    }
                    int b = 0;
                    while (b < 32 && load[b]) ++b;
                    if (b < 32) ++load[b], zb = b;
                    else b = zb >= 0 ? zb : 0;
                    reg[(size_t)(h + l) * kRegSrc + e] = (uint16_t)(kZeroWord | b);
                }
            }
            for (const auto& r : rest)
                if (!r.empty()) return false;  // cannot happen: a lane with no round to spare always takes one
        }
    }
    return true;
}

snp_status snp_batch_load(const snp_desc* descs, int32_t n, const snp_options* opt, snp_batch** out) {
    g_err.clear();
    if (!out) return fail(SNP_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!descs || n < 1) return fail(SNP_ERR_INVALID, "need at least one system");
    const int ct = descs[0].count_type;
    std::vector<snp::BatchSys> sys(n);
    std::vector<long long> row_off(n + 1, 0);
    std::vector<uint32_t> rules, magic, fast, lut;
    std::vector<int> nrp, in_ptr, in_src, slots;
    std::vector<uint16_t> reg_src;  // kRegSrc per slot; system k's from kRegSrc * row_off[k] on
    int m_max = 0, r_max = 0;
    for (int k = 0; k < n; ++k) {
        const snp_desc* d = &descs[k];
        snp_status st = validate(d);
        if (st) return fail(st, "system %d: %s", k, g_err.c_str());
        if (d->count_type != ct) return fail(SNP_ERR_INVALID, "system %d: all systems must share count_type", k);
        if (d->m > 4 * snp::batch_max_threads())
            return fail(SNP_ERR_INVALID, "system %d: m above %d is not supported in batched mode", k,
                        4 * snp::batch_max_threads());
        for (int q = 0; q < d->r; ++q) {
            if (d->rule_i[q] > 255 || d->rule_j[q] > 255 || d->rule_c[q] > 255 || d->rule_p[q] > 255)
                return fail(SNP_ERR_INVALID, "system %d rule %d: batched mode needs i, j, c, p <= 255", k, q);
            if (d->rule_d && d->rule_d[q] != 0)
                return fail(SNP_ERR_INVALID, "system %d rule %d: the batched mode has no delays", k, q);
        }
        snp::BatchSys& B = sys[k];
        B.m = d->m;
        B.r = d->r;
        B.row_off = row_off[k];
        row_off[k + 1] = row_off[k] + d->m;
        B.rule_off = (int)rules.size();
        B.nrp_off = (int)nrp.size();
        B.in_off = (int)in_src.size();
        // Slots: the kernel runs slot s on thread s mod TPB; neurons take the
        // slots in order of decreasing in-degree (ties by index) so that the 64
        // lanes of a wave pull similar numbers of in-synapses.  Rules, tables and
        // in-synapse lists are laid out by slot; perm maps a slot to its neuron
        // (rows in HBM, the H weights).
        std::vector<int> indeg(d->m, 0), perm(d->m), slot_of(d->m);
        for (int e = 0; e < d->n_syn; ++e) indeg[d->syn_dst[e]]++;
        for (int j = 0; j < d->m; ++j) perm[j] = j;
        std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) { return indeg[x] > indeg[y]; });
        for (int s = 0; s < d->m; ++s) slot_of[perm[s]] = s;
        std::vector<int> first(d->m + 1, 0);  // rules of neuron j: [first[j], first[j+1]) (sorted by neuron)
        for (int q = 0; q < d->r; ++q) first[d->rule_neuron[q] + 1]++;
        for (int j = 0; j < d->m; ++j) first[j + 1] += first[j];
        std::vector<int> cnt(d->m + 1, 0), icnt(d->m + 1, 0);
        for (int s = 0; s < d->m; ++s) {
            const int j = perm[s];
            cnt[s + 1] = cnt[s] + first[j + 1] - first[j];
            icnt[s + 1] = icnt[s] + indeg[j];
            for (int q = first[j]; q < first[j + 1]; ++q) {  // the neuron's rules, in their order
                magic.push_back(div_magic((uint32_t)d->rule_j[q]));
                rules.push_back((uint32_t)d->rule_i[q] | ((uint32_t)d->rule_j[q] << 8) |
                                ((uint32_t)d->rule_c[q] << 16) | ((uint32_t)d->rule_p[q] << 24));
            }
        }
        std::vector<int> src(d->n_syn), fill(d->m, 0);
        for (int e = 0; e < d->n_syn; ++e) {
            const int dst = slot_of[d->syn_dst[e]];
            src[icnt[dst] + fill[dst]++] = slot_of[d->syn_src[e]];
        }
        std::vector<uint16_t> reg;
        if (!place_in_synapses(d->m, icnt, src, reg))
            return fail(SNP_ERR_INVALID, "system %d: in-synapse placement left sources unread", k);
        reg_src.insert(reg_src.end(), reg.begin(), reg.end());
        // Tables of the first applicable rule (indexed like nrp: m + 1 entries per
        // system, the last unused), 4 bits per entry: the rule's index in the
        // neuron + 1, 0 for none.  Counts 0-15 by direct lookup (at most 15
        // rules).  For a count n >= T a rule with j = 0 no longer applies
        // (T > max(i, c)) and a rule with j >= 1 applies iff n >= max(i, c)
        // (true) and n = i (mod j); when every such j divides 24 the first
        // applicable rule is a function of n mod 24.
        for (int s = 0; s <= d->m; ++s) {
            const int j = s < d->m ? perm[s] : 0;
            const int q0 = s < d->m ? first[j] : 0, q1 = s < d->m ? first[j + 1] : 0;
            uint32_t T = 0, w[5] = {0, 0, 0, 0, 0};
            const bool small = s < d->m && q1 - q0 <= 15;
            bool ok = small;
            for (int q = q0; ok && q < q1; ++q) {
                const uint32_t ri = (uint32_t)d->rule_i[q], rj = (uint32_t)d->rule_j[q], rc = (uint32_t)d->rule_c[q];
                const uint32_t lo = std::max(ri, rc);
                if (rj == 0) T = std::max(T, lo + 1);
                else {
                    T = std::max(T, lo);
                    if (24 % rj) ok = false;
                }
            }
            for (uint32_t r = 0; ok && r < 24; ++r) {
                uint32_t idx = 0;
                for (int q = q0; q < q1 && !idx; ++q) {
                    const int rj = d->rule_j[q];
                    if (rj > 0 && (((int)r - d->rule_i[q]) % rj + rj) % rj == 0) idx = (uint32_t)(q - q0 + 1);
                }
                w[r / 8] |= idx << (4 * (r % 8));
            }
            for (int n = 0; small && n < 16; ++n) {
                uint32_t idx = 0;
                for (int q = q0; q < q1 && !idx; ++q) {
                    const int ri = d->rule_i[q], rj = d->rule_j[q];
                    const bool in_e = n >= ri && (rj == 0 ? n == ri : (n - ri) % rj == 0);
                    if (in_e && n >= d->rule_c[q]) idx = (uint32_t)(q - q0 + 1);
                }
                w[3 + n / 8] |= idx << (4 * (n % 8));
            }
            fast.push_back((ok ? (T | 0x80000000u) : 0u) | (small ? 0x40000000u : 0u));
            lut.insert(lut.end(), w, w + 5);
            slots.push_back(s < d->m ? j : 0);
        }
        nrp.insert(nrp.end(), cnt.begin(), cnt.end());
        in_ptr.insert(in_ptr.end(), icnt.begin(), icnt.end());
        in_src.insert(in_src.end(), src.begin(), src.end());
        m_max = std::max(m_max, d->m);
        r_max = std::max(r_max, d->r);
    }
    // launch shapes: threads per system and neurons per thread (1, 2 or 4)
    std::vector<std::pair<int, int>> shapes;
    for (int th : {256, 512, 1024}) {
        int npt = (m_max + th - 1) / th;
        npt = npt <= 1 ? 1 : (npt <= 2 ? 2 : (npt <= 4 ? 4 : 0));
        if (npt && snp::batch_lds_bytes(r_max, th, npt) <= 64 * 1024) shapes.push_back({th, npt});
    }
    const int forced = opt ? (int)opt->chunk : 0;
    if (forced) {
        std::vector<std::pair<int, int>> keep;
        for (auto& sh : shapes)
            if (sh.first == forced) keep.push_back(sh);
        if (keep.empty())
            return fail(SNP_ERR_INVALID, "batched mode: %d threads per system do not fit this batch "
                        "(use 256, 512 or 1024, with m <= 4 x threads)", forced);
        shapes = keep;
    }
    if (shapes.empty())
        return fail(SNP_ERR_INVALID, "batched mode: the largest system needs more than 64 KiB of LDS");
    snp_batch* b = new snp_batch();
    b->shapes = shapes;
    b->forced_threads = forced;
    b->n = n;
    b->elem_bytes = ct == SNP_COUNT_U16 ? 2 : 4;
    b->count_max = ct == SNP_COUNT_U16 ? 65535 : INT_MAX;
    b->m_max = m_max;
    b->r_max = r_max;
    b->stream = opt ? (hipStream_t)opt->stream : nullptr;
    b->sys = sys;
    b->row_off = row_off;
#define BLOADCHK(expr)                                                        \
    do {                                                                      \
        hipError_t e_ = (expr);                                               \
        if (e_ != hipSuccess) {                                               \
            delete b;                                                         \
            return fail(SNP_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
        }                                                                     \
    } while (0)
    BLOADCHK(dmalloc(&b->d_sys, sizeof(snp::BatchSys) * n));
    BLOADCHK(dmalloc(&b->d_rules, sizeof(uint32_t) * rules.size()));
    BLOADCHK(dmalloc(&b->d_magic, sizeof(uint32_t) * std::max<size_t>(1, magic.size())));
    BLOADCHK(dmalloc(&b->d_nrp, sizeof(int) * nrp.size()));
    BLOADCHK(dmalloc(&b->d_in_ptr, sizeof(int) * in_ptr.size()));
    BLOADCHK(dmalloc(&b->d_in_src, sizeof(int) * std::max<size_t>(1, in_src.size())));
    BLOADCHK(dmalloc(&b->d_fast, sizeof(uint32_t) * fast.size()));
    BLOADCHK(dmalloc(&b->d_lut, sizeof(uint32_t) * lut.size()));
    BLOADCHK(hipMemcpy(b->d_fast, fast.data(), sizeof(uint32_t) * fast.size(), hipMemcpyHostToDevice));
    BLOADCHK(hipMemcpy(b->d_lut, lut.data(), sizeof(uint32_t) * lut.size(), hipMemcpyHostToDevice));
    BLOADCHK(dmalloc(&b->d_reg_src, sizeof(uint16_t) * reg_src.size()));
    BLOADCHK(hipMemcpy(b->d_reg_src, reg_src.data(), sizeof(uint16_t) * reg_src.size(), hipMemcpyHostToDevice));
    BLOADCHK(dmalloc(&b->d_perm, sizeof(int) * slots.size()));
    BLOADCHK(hipMemcpy(b->d_perm, slots.data(), sizeof(int) * slots.size(), hipMemcpyHostToDevice));
    BLOADCHK(dmalloc(&b->d_halt, sizeof(int) * n));
    BLOADCHK(dmalloc(&b->d_rep, sizeof(int) * n));
    BLOADCHK(dmalloc(&b->d_done, sizeof(int) * n));
    BLOADCHK(dmalloc(&b->d_digest, sizeof(u64) * n));
    BLOADCHK(dmalloc(&b->d_err, sizeof(u64) * n));
    if (!rules.empty()) BLOADCHK(hipMemcpy(b->d_rules, rules.data(), sizeof(uint32_t) * rules.size(), hipMemcpyHostToDevice));
    if (!magic.empty()) BLOADCHK(hipMemcpy(b->d_magic, magic.data(), sizeof(uint32_t) * magic.size(), hipMemcpyHostToDevice));
    BLOADCHK(hipMemcpy(b->d_sys, sys.data(), sizeof(snp::BatchSys) * n, hipMemcpyHostToDevice));
    BLOADCHK(hipMemcpy(b->d_nrp, nrp.data(), sizeof(int) * nrp.size(), hipMemcpyHostToDevice));
    BLOADCHK(hipMemcpy(b->d_in_ptr, in_ptr.data(), sizeof(int) * in_ptr.size(), hipMemcpyHostToDevice));
    if (!in_src.empty())
        BLOADCHK(hipMemcpy(b->d_in_src, in_src.data(), sizeof(int) * in_src.size(), hipMemcpyHostToDevice));
    BLOADCHK(hipStreamCreate(&b->cap_stream));
#undef BLOADCHK
    *out = b;
    return SNP_OK;
}

void snp_batch_free(snp_batch* b) { delete b; }

snp_status snp_batch_offsets(const snp_batch* b, int64_t* offsets) {
    g_err.clear();
    if (!b || !offsets) return fail(SNP_ERR_INVALID, "batch and offsets are required");
    for (int k = 0; k <= b->n; ++k) offsets[k] = b->row_off[k];
    return SNP_OK;
}

snp_status snp_batch_shape(const snp_batch* b, int32_t* threads, int32_t* neurons_per_thread) {
    g_err.clear();
    if (!b || !threads || !neurons_per_thread) return fail(SNP_ERR_INVALID, "batch and outputs are required");
    *threads = b->threads;
    *neurons_per_thread = b->npt;
    return SNP_OK;
}

snp_status snp_batch_run(snp_batch* b, const void* c0_dev, int32_t steps, int32_t detect_repeats, void* final_dev,
                         int32_t* halt_step, int32_t* first_repeat, int32_t* steps_done, uint64_t* digest) {
    g_err.clear();
    if (!b) return fail(SNP_ERR_INVALID, "batch is NULL");
    if (!c0_dev || !final_dev || !halt_step || !first_repeat || !steps_done || !digest)
        return fail(SNP_ERR_INVALID, "c0, final and every result array are required");
    if (steps < 0 || steps > (1 << 24)) return fail(SNP_ERR_INVALID, "steps must be in [0, 2^24]");
    const int interval = snp::batch_interval();
    if (steps > b->cap_steps) {  // checkpoints and H sets sized for this many steps
        if (b->d_ckpt) HIPCHK(hipFree(b->d_ckpt));
        if (b->d_hkey) HIPCHK(hipFree(b->d_hkey));
        if (b->d_hstep) HIPCHK(hipFree(b->d_hstep));
        b->d_ckpt = nullptr;
        b->d_hkey = nullptr;
        b->d_hstep = nullptr;
        b->ckpt_rows = batch_ckpt_rows(steps);
        b->table_slots = batch_table_slots(steps);
        HIPCHK(dmalloc(&b->d_ckpt, (size_t)(b->ckpt_rows * b->row_off[b->n]) * b->elem_bytes));
        HIPCHK(dmalloc(&b->d_hkey, sizeof(u64) * b->table_slots * b->n));
        HIPCHK(dmalloc(&b->d_hstep, sizeof(int) * b->table_slots * b->n));
        b->cap_steps = steps;
    }
    snp::BatchArgs a{b->d_sys, b->d_rules, b->d_magic, b->d_nrp, b->d_in_ptr, b->d_in_src, c0_dev, final_dev, b->d_ckpt,
                     b->ckpt_rows, b->d_hkey, b->d_hstep, b->table_slots, b->m_max, b->r_max, steps,
                     detect_repeats ? 1 : 0, b->count_max, b->d_halt, b->d_rep, b->d_done, b->d_digest, b->d_err};
    a.fast = b->d_fast;
    a.lut = b->d_lut;
    a.perm = b->d_perm;
    a.reg_src = b->d_reg_src;
    auto enqueue = [&](hipStream_t st, int threads, int npt) -> hipError_t {
        if (detect_repeats) {
            const hipError_t e = snp::launch_fill_i32(b->d_hstep, (long long)b->table_slots * b->n, -1, st);
            if (e != hipSuccess) return e;
        }
        return snp::launch_batch_det(b->elem_bytes, threads, npt, a, b->n, st);
    };
    if (!b->threads) {
        // tune once per batch: time every candidate shape on a short run of this batch
        if (b->shapes.size() == 1) {
            b->threads = b->shapes[0].first;
            b->npt = b->shapes[0].second;
        } else {
            hipEvent_t e0, e1;
            HIPCHK(hipEventCreate(&e0));
            HIPCHK(hipEventCreate(&e1));
            snp::BatchArgs trial = a;
            trial.steps = std::min(steps, 2 * interval);
            float best = 0.f;
            hipError_t err = hipSuccess;
            for (auto& sh : b->shapes) {
                float ms = 0.f;
                const snp::BatchArgs keep = a;
                a = trial;
                err = enqueue(b->stream, sh.first, sh.second);  // warm-up
                if (err == hipSuccess) err = hipEventRecord(e0, b->stream);
                if (err == hipSuccess) err = enqueue(b->stream, sh.first, sh.second);
                if (err == hipSuccess) err = hipEventRecord(e1, b->stream);
                if (err == hipSuccess) err = hipEventSynchronize(e1);
                if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
                a = keep;
                if (err != hipSuccess) break;
                if (!b->threads || ms < best) {
                    best = ms;
                    b->threads = sh.first;
                    b->npt = sh.second;
                }
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            HIPCHK(err);
        }
    }
    const snp_batch::Key key{c0_dev, final_dev, steps, detect_repeats ? 1 : 0, b->threads, b->npt, b->cap_steps};
    if (!b->exec || !(key == b->key)) {
        if (b->exec) HIPCHK(hipGraphExecDestroy(b->exec));
        b->exec = nullptr;
        hipGraph_t graph = nullptr;
        HIPCHK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
        const hipError_t le = enqueue(b->cap_stream, b->threads, b->npt);
        const hipError_t ce = hipStreamEndCapture(b->cap_stream, &graph);
        HIPCHK(le);
        HIPCHK(ce);
        const hipError_t ie = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHK(ie);
        b->key = key;
    }
    HIPCHK(hipGraphLaunch(b->exec, b->stream));
    std::vector<u64> err(b->n);
    HIPCHK(hipMemcpyAsync(halt_step, b->d_halt, sizeof(int) * b->n, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipMemcpyAsync(first_repeat, b->d_rep, sizeof(int) * b->n, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipMemcpyAsync(steps_done, b->d_done, sizeof(int) * b->n, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipMemcpyAsync(digest, b->d_digest, sizeof(u64) * b->n, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipMemcpyAsync(err.data(), b->d_err, sizeof(u64) * b->n, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    for (int k = 0; k < b->n; ++k) {
        if (err[k] & 1) return fail(SNP_ERR_OVERFLOW, "system %d: a count left the count type's range", k);
        if (err[k] & 2)
            return fail(SNP_ERR_DEVICE, "system %d: two configurations share a 64-bit hash; repeat detection "
                        "cannot vouch for its answer", k);
    }
    return SNP_OK;
}

// snp_run_batch: the handles' systems packed into one batch, kept while the
// list of handles (by id) stays the same.  The packed rows live in buffers of
// their own, so the batch's recorded graph is replayed across calls.
namespace {
struct RunBatchCache {
    std::vector<unsigned long long> uids;
    snp_batch* b = nullptr;
    int n = 0, elem_bytes = 4;
    void* d_c0 = nullptr;        // packed C0 rows
    void* d_fin = nullptr;       // packed final rows
    void** d_ptrs = nullptr;     // [2n]: C0 sources, then final destinations
    long long* d_off = nullptr;  // [n + 1] element offsets of the packed rows
    std::vector<void*> h_ptrs;
    void release() {
        if (b) snp_batch_free(b);
        void* ps[] = {d_c0, d_fin, d_ptrs, d_off};
        for (void* p : ps)
            if (p) (void)hipFree(p);
        *this = RunBatchCache{};
    }
};
// One per thread; its device buffers are replaced when the list of handles
// changes and otherwise live until the process ends.
thread_local RunBatchCache* g_rb = nullptr;
}  // namespace

snp_status snp_run_batch(snp_system* const* systems, int32_t n, const void* const* c0_dev, int32_t steps,
                         void* const* final_dev, int32_t* halt_step, int32_t* first_repeat_step,
                         uint64_t* trajectory_digest) {
    g_err.clear();
    if (!systems || n < 1 || !c0_dev || !final_dev || !halt_step || !first_repeat_step || !trajectory_digest)
        return fail(SNP_ERR_INVALID, "systems, c0_dev, final_dev and every result array are required (n >= 1)");
    for (int k = 0; k < n; ++k) {
        if (!systems[k]) return fail(SNP_ERR_INVALID, "system %d is NULL", k);
        if (systems[k]->track >= 0)
            return fail(SNP_ERR_INVALID, "system %d follows an output neuron: the batched mode does not", k);
        if (systems[k]->delays)
            return fail(SNP_ERR_INVALID, "system %d has rules with delays: the batched mode has none", k);
        if (!c0_dev[k] || !final_dev[k]) return fail(SNP_ERR_INVALID, "system %d: c0 or final is NULL", k);
        if (systems[k]->count_type != systems[0]->count_type)
            return fail(SNP_ERR_INVALID, "system %d: all systems must share one count type", k);
    }
    if (!g_rb) g_rb = new RunBatchCache();
    RunBatchCache& C = *g_rb;
    std::vector<unsigned long long> uids(n);
    for (int k = 0; k < n; ++k) uids[k] = systems[k]->uid;
    hipStream_t st = systems[0]->stream;
    if (uids != C.uids || !C.b) {
        C.release();
        std::vector<snp_desc> descs(n);
        for (int k = 0; k < n; ++k) {
            const snp_system* S = systems[k];
            descs[k] = snp_desc{S->m, S->r, S->h_rn.data(), S->h_ri.data(), S->h_rj.data(), S->h_rc.data(),
                                S->h_rp.data(), (int32_t)S->h_ss.size(), S->h_ss.data(), S->h_sd.data(), nullptr,
                                S->count_type};
        }
        snp_options o{};
        o.max_rows = 1;
        o.stream = st;
        snp_status r = snp_batch_load(descs.data(), n, &o, &C.b);
        if (r) return r;
        C.n = n;
        C.elem_bytes = C.b->elem_bytes;
        const long long total = C.b->row_off[n];
        HIPCHK(dmalloc(&C.d_c0, (size_t)std::max<long long>(1, total) * C.elem_bytes));
        HIPCHK(dmalloc(&C.d_fin, (size_t)std::max<long long>(1, total) * C.elem_bytes));
        HIPCHK(dmalloc(&C.d_ptrs, sizeof(void*) * 2 * n));
        HIPCHK(dmalloc(&C.d_off, sizeof(long long) * (n + 1)));
        HIPCHK(hipMemcpy(C.d_off, C.b->row_off.data(), sizeof(long long) * (n + 1), hipMemcpyHostToDevice));
        C.h_ptrs.assign(2 * n, nullptr);
        C.uids = uids;
    }
    for (int k = 0; k < n; ++k) {
        C.h_ptrs[k] = const_cast<void*>(c0_dev[k]);
        C.h_ptrs[n + k] = final_dev[k];
    }
    HIPCHK(hipMemcpyAsync(C.d_ptrs, C.h_ptrs.data(), sizeof(void*) * 2 * n, hipMemcpyHostToDevice, st));
    HIPCHK(snp::launch_pack_rows((void* const*)C.d_ptrs, C.d_off, C.d_c0, n, C.elem_bytes, true, st));
    std::vector<int32_t> done(n);
    snp_status r = snp_batch_run(C.b, C.d_c0, steps, 1, C.d_fin, halt_step, first_repeat_step, done.data(),
                                 trajectory_digest);
    if (r) return r;
    HIPCHK(snp::launch_pack_rows((void* const*)(C.d_ptrs + n), C.d_off, C.d_fin, n, C.elem_bytes, false, st));
    HIPCHK(hipStreamSynchronize(st));
    return SNP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// snp_batch_run_static: the deterministic batched run with every scratch
// buffer (per-system results, checkpoint rows, H sets) carved from one
// file-scope device array, so that the call allocates nothing.  Each device
// the library runs on holds its own copy of the array until the process ends;
// its address is looked up once per device and kept.
// ---------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device (the array's name in host
// code is not a device address).
snp_status static_scratch(unsigned char** out) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SNP_ERR_DEVICE, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(SNP_ERR_DEVICE, "no device address for the static scratch array");
        g_scratch_dev[dev] = p;
    }
    *out = (unsigned char*)g_scratch_dev[dev];
    return SNP_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

extern "C" snp_status snp_batch_run_static(snp_batch* b, const void* c0_dev, int32_t steps, int32_t detect_repeats,
                                           void* final_dev, int32_t* halt_step, int32_t* first_repeat,
                                           int32_t* steps_done, uint64_t* digest) {
    g_err.clear();
    if (!b) return fail(SNP_ERR_INVALID, "batch is NULL");
    if (!c0_dev || !final_dev || !halt_step || !first_repeat || !steps_done || !digest)
        return fail(SNP_ERR_INVALID, "c0, final and every result array are required");
    if (steps < 0 || steps > (1 << 24)) return fail(SNP_ERR_INVALID, "steps must be in [0, 2^24]");
    const int n = b->n;
    const long long rows = batch_ckpt_rows(steps);
    const u64 slots = batch_table_slots(steps);
    // layout: halt, first repeat, steps done (int32 each), digest, error bits
    // (uint64 each), checkpoint rows, then the H sets (repeat detection only)
    size_t o = 0;
    const size_t o_halt = o;
    o = align256(o + sizeof(int) * n);
    const size_t o_rep = o;
    o = align256(o + sizeof(int) * n);
    const size_t o_done = o;
    o = align256(o + sizeof(int) * n);
    const size_t o_dig = o;
    o = align256(o + sizeof(u64) * n);
    const size_t o_err = o;
    o = align256(o + sizeof(u64) * n);
    const size_t o_ckpt = o;
    o = align256(o + (size_t)(rows * b->row_off[n]) * b->elem_bytes);
    const size_t o_hstep = o, o_hkey = align256(o + sizeof(int) * slots * n);
    if (detect_repeats) o = align256(o_hkey + sizeof(u64) * slots * n);
    if (o > kStaticScratchBytes)
        return fail(SNP_ERR_CAPACITY, "snp_batch_run_static: %d systems x %d steps need %zu bytes of scratch, above "
                    "the static %zu (use snp_batch_run, or fewer systems or steps)", n, steps, o,
                    kStaticScratchBytes);
    unsigned char* base = nullptr;
    snp_status st = static_scratch(&base);
    if (st) return st;
    // launch shape: the one an earlier snp_batch_run tuned, else the widest that fits
    // (timing candidates would create events)
    int threads = b->threads, npt = b->npt;
    if (!threads) {
        threads = b->shapes.back().first;
        npt = b->shapes.back().second;
    }
    int* d_halt = (int*)(base + o_halt);
    int* d_rep = (int*)(base + o_rep);
    int* d_done = (int*)(base + o_done);
    u64* d_dig = (u64*)(base + o_dig);
    u64* d_err = (u64*)(base + o_err);
    int* d_hstep = (int*)(base + o_hstep);
    snp::BatchArgs a{b->d_sys, b->d_rules, b->d_magic, b->d_nrp, b->d_in_ptr, b->d_in_src, c0_dev, final_dev,
                     base + o_ckpt, rows, (u64*)(base + o_hkey), d_hstep, slots, b->m_max, b->r_max, steps,
                     detect_repeats ? 1 : 0, b->count_max, d_halt, d_rep, d_done, d_dig, d_err};
    a.fast = b->d_fast;
    a.lut = b->d_lut;
    a.perm = b->d_perm;
    a.reg_src = b->d_reg_src;
    // every result is written by the kernel; the H sets start empty (-1), cleared by a fill kernel
    if (detect_repeats) HIPCHK(snp::launch_fill_i32(d_hstep, (long long)slots * n, -1, b->stream));
    HIPCHK(snp::launch_batch_det(b->elem_bytes, threads, npt, a, n, b->stream));
    HIPCHK(hipMemcpyAsync(halt_step, d_halt, sizeof(int) * n, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipMemcpyAsync(first_repeat, d_rep, sizeof(int) * n, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipMemcpyAsync(steps_done, d_done, sizeof(int) * n, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipMemcpyAsync(digest, d_dig, sizeof(u64) * n, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    // the error bits, 64 systems per copy into a buffer on the stack
    for (int k0 = 0; k0 < n; k0 += 64) {
        u64 e[64];
        const int cnt = std::min(64, n - k0);
        HIPCHK(hipMemcpy(e, d_err + k0, sizeof(u64) * cnt, hipMemcpyDeviceToHost));
        for (int q = 0; q < cnt; ++q) {
            if (e[q] & 1) return fail(SNP_ERR_OVERFLOW, "system %d: a count left the count type's range", k0 + q);
            if (e[q] & 2)
                return fail(SNP_ERR_DEVICE, "system %d: two configurations share a 64-bit hash; repeat detection "
                            "cannot vouch for its answer", k0 + q);
        }
    }
    return SNP_OK;
}
