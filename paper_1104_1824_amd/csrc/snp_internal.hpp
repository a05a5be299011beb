// Internal interface between the C-ABI runtime (snp_api.hip) and the gfx950
// kernels (snp_kernels.hip).  Not installed, not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace snp {

typedef unsigned long long u64;

// Saturation point of child counts Psi and of their prefix sums (2^62): every
// count at or above it is "too many to enumerate", and sums of two such values
// still fit in 64 bits.
constexpr u64 kPsiSat = 1ULL << 62;

// Visited-set entry: high 32 bits = hash tag, low 32 bits = row reference.
// References below kStageBase name rows of the row store (the configurations
// recorded so far); kStageBase + b names child b of the chunk being expanded.
constexpr uint32_t kStageBase = 0x80000000u;
constexpr uint32_t kMaxChunk = 1u << 30;
constexpr u64 kEmpty = ~0ULL;           // never a valid entry (reference 0xFFFFFFFF)
constexpr u64 kTomb = ~0ULL - 1;        // removed entry (reference 0xFFFFFFFE); never reused
// Children per tile of the chunk-wide scans (new-child flags, offsets).
constexpr int kScanTile = 1024;

// Device counters one expansion pass reads back in a single copy.
struct DevCounters {
    u64 halting;       // parents with no applicable rule
    u64 overflow;      // nonzero: a child count left the type's range
    u64 probe_fail;    // nonzero: a probe sequence found no free slot
    u64 cap_g;         // chunk-relative index + 1 of the child that filled the cap (0: none)
    u64 tombs;         // entries turned into tombstones by this pass
    u64 total;         // scan total (children of the frontier / new children of a chunk)
    u64 ncand;         // children whose probe met an entry with their tag (row compare pending)
    u64 cap_par;       // parent (frontier index) of the child that filled the cap
    u64 count;         // scratch count (halting parents of a frontier prefix)
    u64 beff;          // children the chunk really covers: min(B, children of the prefix - g0)
    u64 psi_total;     // canonical children of the frontier prefix after this pass's extension
    u64 c0_bad;        // walk start: C0 holds a count outside the count type's range
    u64 collisions;    // probes that met an entry with their tag whose row differed
    u64 mfma;          // int8 matrix-core instructions issued (16x16x64 each)
    u64 psif_lo;       // all children (every valid spiking vector) of the parents this pass
    u64 psif_hi;       //   added to the prefix: sum of (Psi mod 2^31) and of (Psi >> 31)
    u64 cap_t;         // child index t of the child that filled the cap
    u64 capf_lo;       // all children of the parents before the cap child's parent, split
    u64 capf_hi;       //   as psif_lo / psif_hi
    u64 tend;          // canonical children the chunks may take: the prefix's, or fewer where
                       // the child budget ends (the budget's clip)
    u64 bud_par;       // budget clip: parent of the last child within the budget, + 1 (0: none)
    u64 verify_fail;   // keys-first pass: a child taken for a repeat (its key met an entry) has a
                       // row that differs from that entry's; the pass is redone with staged rows
};

// Device-side description of a loaded system.
struct DevSystem {
    int m, r;
    const int* nrule_ptr;  // [m+1] rules of neuron n: nrule_ptr[n] .. nrule_ptr[n+1]
    const int4* rules;     // [r] (i, j, c, p) (with delays, p | (d << 16) in the last)
    const int* in_ptr;     // [m+1] in-synapses of neuron d: in_src[in_ptr[d] .. in_ptr[d+1])
    const int* in_src;     // sources of the in-synapses
    int nnz_in;            // number of synapses
    const int8_t* M8;      // [r*m] int8 copy of M_Pi (nullptr when some |entry| > 127)
    long long count_max;
    const u64* R;          // [m] hash weights: R[n] = mix64((n + 1) * gamma)
    const u64* hM;         // [r] H of every row of M_Pi (entries sign-extended, mod 2^64)
    int max_in;            // largest in-degree of a neuron
    const int* in_lane;    // [16 * 64] in-synapse e of neuron j at e * 64 + j (-1: none),
                           // filled when m <= 64 and max_in <= 16
    u64 psi_cap;           // largest Psi of a parent: 1 in deterministic mode (first spiking
                           // vector only), kPsiSat otherwise
    int track;             // >= 0: rows end with the output neuron's spike train, the spikes
                           // sent to the environment (at most 2 counted) at column track and
                           // the steps from the first to the second at track + 1; the m
                           // above counts these two columns (neurons without rules or synapses)
    int out;               // the output neuron (with track >= 0)
    // Delays.  The first mcount columns of a row are spike counts; with delays
    // every neuron owning a rule with a delay has two more columns from dfirst
    // on: wait (steps until it sends its delayed spikes, 0: open) and pend
    // (the spikes it will send).  dlink[j], j < mcount: column of neuron j's
    // wait (-1: none); dlink[c], c >= dfirst: the neuron whose state column c
    // holds.  rules[k].w then holds p | (d << 16).  dlink null: no delays
    // (rules[k].w = p).
    const int* dlink;
    int mcount;
    int dfirst;
};

// One chunk of canonical children [g0, g0 + B) of the frontier (canonical
// children numbered parent by parent, each parent's in child-index order).
struct ChunkArgs {
    const void* frontier;  // n rows
    long long n;
    const u64* psi;        // [n] canonical children per parent (0: none)
    const u64* off;        // [n] exclusive prefix sums of psi
    u64 g0;
    long long B;
    void* stage;           // [B] child rows
    u64* hash;             // [B]
    int* cpar;             // [B] parent index p in the frontier
    u64* ct;               // [B] child index t within the parent (Algorithm 2 II-3 order)
    u64 hash_mask;
    DevCounters* ctr;
    const u64* Tdev;       // canonical children the chunks may take: the chunk stops there
    int kmax;              // int8 form: most rule columns a segment may put on the matrix cores
    int tiles;             // int8 form: consecutive 64-child tiles per workgroup (0: automatic)
    int run;               // sparse form: consecutive children per wave (0: automatic)
    // visited-set probe done by the expansion itself (the one-neuron-per-lane
    // form); null table: the probe runs as a kernel of its own
    u64* table;
    u64 slot_mask;
    uint32_t* slot;        // [B]
    uint32_t* cand;        // [B]
    // Keys-first passes of the int8 form.  mode 0 stages every child's row
    // (then probe, row compares, commit copy); mode 1 computes keys, parents and
    // child indices only; mode 2 computes the rows once the new children are
    // known: new child b with prefix q = tile_pre[b / kScanTile] + pos[b] below
    // limit_new goes to row arena_row + q of the row store, every other child
    // to its stage row.
    int mode;
    const uint32_t* flag;
    const uint32_t* pos;
    const uint32_t* tile_pre;
    void* arena;
    long long arena_row;
    long long limit_new;
};

// Insert/commit arguments.
struct TableArgs {
    u64* table;
    u64 slot_mask;
    const void* arena;     // row store (rows referenced by entries below kStageBase)
    const void* stage;
    const u64* hash;
    uint32_t* slot;        // [B] slot each child resolved to
    long long B;
    DevCounters* ctr;
    uint32_t* cand;        // [B] children waiting for a row compare
    int direct;            // keys-first pass: an entry with the child's tag is taken as its
                           // configuration (the earliest child keeps an entry of the chunk);
                           // no row compare (the rows are checked after the row pass)
};

// Row check of a keys-first pass: rows and destinations as in ChunkArgs mode 2.
struct VerifyArgs {
    const u64* table;
    const uint32_t* slot;
    const void* stage;
    const void* arena;
    const uint32_t* flag;
    const uint32_t* pos;
    const uint32_t* tile_pre;
    long long arena_row;
    long long limit_new;
    long long B;
    DevCounters* ctr;
};

struct CommitArgs {
    const u64* table_ro;
    u64* table;
    const uint32_t* slot;
    const u64* hash;
    const uint32_t* pos;   // [B] exclusive scan of the new-child flags within each scan tile
    const uint32_t* flag;  // [B] 1: child is the first occurrence of a new configuration
    const uint32_t* tile_sums;  // [tiles] flags of every scan tile
    const uint32_t* tile_pre;   // [tiles] exclusive scan of tile_sums (filled only for many tiles)
    const void* stage;
    const int* cpar;
    const u64* ct;
    const u64* psif;       // [n] all children of every parent (the cap child's index g)
    long long B;
    void* arena;           // row store
    long long level_base;  // row-store index of the level's first row
    long long level_count; // rows of the level recorded before this chunk
    long long limit;       // most rows the level may hold
    void* row2;            // nullable second destination (index level_count + pos)
    long long* par_out;    // nullable parent index output
    long long par_out_base;
    long long par_value_base;
    long long* t_out;      // nullable child index output
    uint32_t* row_slot;    // [max_rows] slot of every row-store row
    DevCounters* ctr;
    const uint8_t* hflag;  // nullable halting flags of the frontier: the block that fills the
                           // cap counts them up to the cap child's parent into ctr->count, and
                           // sums psif before that parent into ctr->capf_lo / capf_hi
    int copy;              // 1: copy the new rows from the stage; 0: they are in place (keys-first)
};

// Deterministic batched run: one system per workgroup.
struct BatchSys {
    int m, r;
    long long row_off;      // first element of the system's row in packed row buffers
    int rule_off;           // first packed rule of the system
    int nrp_off;            // first entry of the system's (m+1)-long rule and in-synapse offsets
    int in_off;             // first in-synapse source of the system
};

struct BatchArgs {
    const BatchSys* sys;
    const uint32_t* rules;  // packed (i | j << 8 | c << 16 | p << 24)
    const uint32_t* magic;  // per rule: multiplier for an exact (n - i) / j (j >= 2; 0 otherwise)
    const int* nrp;         // per system: rules of slot s are [nrp[s], nrp[s+1]) (system-relative)
    const int* in_ptr;      // per system: in-synapses of slot s are in_src[in_off + in_ptr[s] ..)
    const int* in_src;      // source slots
    const void* c0;
    void* final_out;
    void* ckpt;             // system k's checkpoint rows (m elements each, by slot) start at element
                            // ckpt_rows * row_off of system k
    long long ckpt_rows;    // checkpoint rows per system
    u64* hkey;              // system k's H set: slots k * table_slots .. + table_slots
    int* hstep;
    u64 table_slots;        // per system, power of two
    int m_max, r_max;
    int steps;
    int detect_repeats;
    long long count_max;
    int* halt_step;
    int* first_repeat;
    int* steps_done;
    u64* digest;
    u64* err;               // bit 0: overflow; bit 1: two configurations with one 64-bit H
    // Per slot (indexed like nrp; the arrays above are laid out by slot too):
    // tables of the first applicable rule.  fast = T | ok << 31 | small << 30:
    // for a count n >= T every rule with j = 0 is past its only count and every
    // other one applies iff n = i (mod j), so with ok (every j divides 24 and at
    // most 15 rules) the first applicable rule depends on n mod 24 alone;
    // lut[5 k .. 5 k + 2] hold 4 bits per residue: the rule's index in the
    // neuron + 1 (0: none); with small (at most 15 rules) lut[5 k + 3 .. 5 k + 4]
    // hold the same for the counts 0-15.
    const uint32_t* fast;
    const uint32_t* lut;
    const int* perm;        // per slot: its neuron (the entry in c0 and final_out rows, H weight)
    // Per slot (system k's from 32 * row_off on): the slot whose production
    // word each of the 32 pull rounds reads, or 0xFFE0 | b for the zero word
    // in bank b (placed at load so that a half-wave's reads in a round fall on
    // distinct LDS banks where possible); the sources past the first 32 of a
    // slot are read from the end of its in_src list.
    const uint16_t* reg_src;
};

size_t batch_lds_bytes(int r_max, int threads, int npt);
int batch_max_threads();
int batch_interval();
hipError_t launch_batch_det(int elem_bytes, int threads, int npt, const BatchArgs& a, int n_sys, hipStream_t st);
hipError_t launch_fill_i32(int* p, long long n, int v, hipStream_t st);
// Copy n rows between separate buffers (ptrs[k]) and one packed buffer (row k at
// element off[k] .. off[k+1]); to_packed selects the direction.  ptrs and off
// are device arrays.
hipError_t launch_pack_rows(void* const* ptrs, const long long* off, void* packed, int n, int elem_bytes,
                            bool to_packed, hipStream_t st);

// Per parent: canonical children (psi), all children (psif), halting flag;
// the sum of psif goes to ctr->psif_lo / psif_hi, the halting parents to ctr->halting.
hipError_t launch_psi(int elem_bytes, const DevSystem& s, const void* frontier, long long n,
                      long long expand_max, u64* psi, u64* psif, uint8_t* halt_flag, DevCounters* ctr,
                      hipStream_t st);
bool psi_scan_fits(const DevSystem& s, long long n);  // launch_psi_scan_small takes n parents (m <= 64)
// launch_psi and the offsets of the canonical counts of n (psi_scan_fits)
// parents in one launch; offsets start at *base_dev (nullable: 0); the new
// total goes to *total_dev and ctr->psi_total.
hipError_t launch_psi_scan_small(int elem_bytes, const DevSystem& s, const void* frontier, long long n,
                                 long long expand_max, u64* psi, u64* psif, uint8_t* halt_flag, u64* off,
                                 const u64* base_dev, u64* total_dev, DevCounters* ctr, hipStream_t st);
// Child budget: the canonical children of the prefix [0, n) whose index g among
// all children is below `budget`; *tend = min(*total, that count), ctr->tend
// likewise, ctr->bud_par = parent of child budget - 1, plus 1 (0 when the
// prefix holds no more than budget children).
hipError_t launch_budget_clip(int elem_bytes, const DevSystem& s, const void* frontier, long long n,
                              const u64* psif, const u64* off, const u64* total, u64 budget, u64* tend,
                              DevCounters* ctr, hipStream_t st);
hipError_t launch_scan_u64(const u64* in, u64* out, long long n, u64* tile_sums, u64* tile_pre,
                           u64* total, const u64* base_dev, u64* total_copy, hipStream_t st);
hipError_t launch_count_flags(const uint8_t* flags, long long n, u64* out, hipStream_t st);
hipError_t launch_count_flags_cap(const uint8_t* flags, const u64* psif, long long n, DevCounters* ctr,
                                  hipStream_t st);
long long scan_tiles(long long n);
hipError_t launch_expand_int8(int elem_bytes, const DevSystem& s, const ChunkArgs& a, hipStream_t st);
size_t int8_lds(int m, int nt);
// *probed: the launch also probed the visited set for every child (a.table set)
hipError_t launch_expand_sparse(int elem_bytes, const DevSystem& s, const ChunkArgs& a, hipStream_t st,
                                bool* probed);
// probe false: the children were probed by the expansion; only the row compares run
hipError_t launch_insert(int elem_bytes, int m, const TableArgs& a, hipStream_t st, bool probe);
// scan: always fill tile_pre (else only past kCommitTiles tiles, the commit summing them itself)
hipError_t launch_flags(const u64* table, const uint32_t* slot, long long B, DevCounters* ctr, uint32_t* flag,
                        uint32_t* pos, uint32_t* tile_sums, uint32_t* tile_pre, hipStream_t st, bool scan = false);
hipError_t launch_verify(int elem_bytes, int m, const VerifyArgs& a, hipStream_t st);
hipError_t launch_commit(int elem_bytes, int m, const CommitArgs& a, hipStream_t st);
hipError_t launch_fill_u64(u64* p, long long n, u64 v, hipStream_t st);
hipError_t launch_start_walk(int elem_bytes, int m, const u64* R, u64* table, u64 slot_mask, const void* c0,
                             void* arena, long long count_max, u64 hash_mask, uint32_t* row_slot, DevCounters* sc,
                             long long* par0, long long* chi0, const DevSystem& s, long long expand_max, u64* psi0,
                             u64* psif0, uint8_t* hflag0, u64* off0, u64* Tdev, hipStream_t st);
hipError_t launch_rows_insert(int elem_bytes, int m, const u64* R, u64* table, u64 slot_mask, const void* arena,
                              long long first, long long count, u64 hash_mask, uint32_t* row_slot,
                              DevCounters* ctr, hipStream_t st);
hipError_t launch_rollback(const uint32_t* row_slot, u64* table, long long first, long long count,
                           hipStream_t st);

}  // namespace snp
