// gfx950 kernel of the deterministic single-branch run of many independent
// SN P systems in one launch: at every step each neuron fires the first of its
// applicable rules (Section 2.1: one rule per neuron, all neurons on a global
// clock; the first of Algorithm 2's spiking vectors), C_{k+1} = C_k + S_k.M
// (Equation next-config), until the step limit or a halting configuration.
//
// One workgroup of TPB threads runs one system; thread t owns slots
// t, t + TPB, ... (NPT per thread), each holding one neuron (neurons take the
// slots by decreasing in-degree, so a wave's in-synapse pulls are alike); a
// slot past m runs as a neuron with no rule, no in-synapse and weight 0, so
// the step has no per-lane branch.
// Counts, rule tables and the LDS addresses of the first kInReg in-synapse
// sources of every owned neuron live in registers; the block shares the packed
// rule table and double-buffered production words in LDS.  A step: every
// neuron writes the production p of its fired rule (0: none), one barrier
// (which also tells whether any neuron fired), then every neuron pulls
// C' = C - c + sum of p over its in-synapses, in rounds of one LDS read per
// lane whose sources were placed at load so that a half-wave's reads in a round
// fall on distinct banks (a lane with nothing to read takes a zero word in a
// free bank).  Step k uses buffer k & 1, so
// the barrier of step k+1 separates step k's reads from step k+2's writes; the
// two buffers sit a fixed distance apart at the start of LDS and the step loop
// is unrolled by parity, so the odd buffer is reached through the LDS
// instruction's offset field.  TPB and NPT are picked per batch by timing the
// candidates (host side).
//
// Trajectory checksum: H(C) = sum_n C[n] * R_n (mod 2^64) with R_n the
// SplitMix64 stream (seed 0); digest = sum_k mix64(H(C_k) + k * gamma).  Each
// wave sums its lanes' terms of 4 steps at once (a transposed butterfly: the
// first two stages halve the number of values per lane, so 4 sums cost about
// what one plain wave sum costs), leaving one partial sum per wave and step in
// LDS; the block adds them up once every kBatch steps.  First repeat: at those
// boundaries the block stores a checkpoint row and looks the batch's H values
// up in a per-system open-addressing set of earlier H values (and within the
// batch); a candidate pair (l, k) is confirmed by re-simulating C_l and C_k
// from their checkpoints and comparing the rows.  A candidate whose rows differ (two
// configurations with one 64-bit H) is reported as an error, never guessed.
#include "snp_internal.hpp"

namespace snp {

namespace {

constexpr int kInReg = 32;     // in-synapses per neuron held in registers
constexpr int kBatch = 64;     // steps between checkpoints / repeat checks (a multiple of 4)
constexpr int kGroup = 4;      // steps per wave sum of the H terms
constexpr int kZeros = 32;     // zero words after the slots of a production buffer, one per LDS bank
constexpr int kMaxThreads = 1024;
constexpr u64 kGamma = 0x9E3779B97F4A7C15ULL;

__device__ __forceinline__ u64 mix64(u64 z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// 64-bit wave sum on DPP: row shifts 1, 2, 4, 8 then row broadcasts of lanes
// 15 and 31; lane 63 holds the total, returned to every lane.
#define SNP_DPP64(V, CTRL, RM, BC)                                                                \
    do {                                                                                          \
        const uint32_t lo_ = __builtin_amdgcn_update_dpp(0u, (uint32_t)(V), CTRL, RM, 0xf, BC);    \
        const uint32_t hi_ = __builtin_amdgcn_update_dpp(0u, (uint32_t)((V) >> 32), CTRL, RM, 0xf, BC); \
        (V) += ((u64)hi_ << 32) | lo_;                                                            \
    } while (0)

__device__ __forceinline__ u64 wave_sum64(u64 v) {
    SNP_DPP64(v, 0x111, 0xf, true);
    SNP_DPP64(v, 0x112, 0xf, true);
    SNP_DPP64(v, 0x114, 0xf, true);
    SNP_DPP64(v, 0x118, 0xf, true);
    SNP_DPP64(v, 0x142, 0xa, false);
    SNP_DPP64(v, 0x143, 0xc, false);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, 63);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), 63);
    return ((u64)hi << 32) | lo;
}
#undef SNP_DPP64

template <int CTRL>
__device__ __forceinline__ u64 dpp64(u64 v) {
    const uint32_t lo = __builtin_amdgcn_update_dpp(0u, (uint32_t)v, CTRL, 0xf, 0xf, false);
    const uint32_t hi = __builtin_amdgcn_update_dpp(0u, (uint32_t)(v >> 32), CTRL, 0xf, 0xf, false);
    return ((u64)hi << 32) | lo;
}

// One transposed butterfly stage over a lane bit: a lane keeps x (bit clear)
// or y (bit set) and adds the partner's other one; the partner (CTRL) differs
// from the lane in that bit only.
template <int CTRL>
__device__ __forceinline__ u64 tstage(u64 x, u64 y, bool bit) {
    return (bit ? y : x) + dpp64<CTRL>(bit ? x : y);
}

// t + the same lane's t in the other row of its row pair (lanes 16 apart) or
// in the other half of the wave (lanes 32 apart): the permlane swaps of a value
// with itself leave, in each lane, its own and its partner's value.
__device__ __forceinline__ u64 xor_sum16(u64 t) {
    const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)t, (uint32_t)t, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(t >> 32), (uint32_t)(t >> 32), false, false);
    return (((u64)hi[0] << 32) | lo[0]) + (((u64)hi[1] << 32) | lo[1]);
}
__device__ __forceinline__ u64 xor_sum32(u64 t) {
    const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)t, (uint32_t)t, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(t >> 32), (uint32_t)(t >> 32), false, false);
    return (((u64)hi[0] << 32) | lo[0]) + (((u64)hi[1] << 32) | lo[1]);
}

// Wave sums of four per-lane values at once: lane l returns the sum over the
// wave's 64 lanes of h[l & 3].  Stages: lane bit 0 (quad_perm 1,0,3,2) and bit 1
// (quad_perm 2,3,0,1) transposed, leaving the quad's sum of h[l & 3]; then
// the quads of a row (row_ror 4, then row_ror 8: every quad of the row reaches
// every lane), then the rows (lanes 16 apart, then 32 apart; VALU swaps, no LDS).
__device__ __forceinline__ u64 wave_sum4(const u64 (&h)[kGroup], int lane) {
    const u64 r0 = tstage<0xB1>(h[0], h[1], lane & 1), r1 = tstage<0xB1>(h[2], h[3], lane & 1);
    u64 t = tstage<0x4E>(r0, r1, (lane >> 1) & 1);
    t += dpp64<0x124>(t);
    t += dpp64<0x128>(t);
    return xor_sum32(xor_sum16(t));
}

typedef __attribute__((address_space(3))) int lds_i32;

// A generic pointer into LDS as an LDS byte address, and a load from one.
__device__ __forceinline__ uint32_t lds_addr(const void* p) { return (uint32_t)(uintptr_t)(const lds_i32*)p; }
__device__ __forceinline__ int lds_load(uint32_t addr) { return *(const lds_i32*)(uintptr_t)addr; }

// Packed rule (i | j << 8 | c << 16 | p << 24): a^n in L(a^i (a^j)*) and n >= c.
// (n - i) mod j by the exact multiply-shift quotient with the rule's
// multiplier M (Granlund-Montgomery; every 32-bit x, 2 <= j < 256); no branch.
__device__ __forceinline__ bool applies_packed(int n, uint32_t R, uint32_t M) {
    const int i = R & 0xFF, j = (R >> 8) & 0xFF, c = (R >> 16) & 0xFF;
    const uint32_t x = (uint32_t)(n - i);
    const uint32_t l = 32u - (uint32_t)__clz(max(j, 2) - 1);
    const uint32_t t = __umulhi(M, x);
    const uint32_t q = (t + ((x - t) >> 1)) >> (l - 1);
    const bool mod0 = j == 0 ? x == 0 : (j == 1 ? true : x == q * (uint32_t)j);
    return n >= i && n >= c && mod0;
}

template <int NPT>
struct Neurons {
    int cnt[NPT];          // current spike count
    int T[NPT];            // counts from T on take the residue table (0x7FFFFFFF: never)
    int S[NPT];            // counts below S take the small-count table (16, or 0: never)
    uint32_t l0[NPT], l1[NPT], l2[NPT];  // first applicable rule + 1 per count mod 24, 4 bits each
                                         // (residues 0-7, 8-15, 16-23; named, never indexed)
    uint32_t s0[NPT], s1[NPT];           // the same per count 0-7 and 8-15
    u64 cpw[NPT];          // (c | p << 8) of the neuron's rules 1-3 at bits 16 k (k = 1-3; bits 0-15: 0)
    bool far[NPT];         // uniform: a lane of the wave has more than 3 rules
    bool slow[NPT];        // uniform: a lane of the wave has counts that neither table covers
    int orig[NPT];         // the slot's neuron (its entry in rows of HBM)
    int rs[NPT], rn[NPT];  // rules: lrules[rs .. rs + rn)
    int rw[NPT];           // the wave's largest rule count (uniform)
    int is[NPT], in[NPT];  // in-synapse sources: in_src[is .. is + in)
    uint32_t src[NPT][kInReg];  // LDS addresses in the even buffer of the first kInReg sources
                                // (the zero slot past in)
    int kw[NPT];           // the wave's largest in-degree held in registers (uniform)
    u64 R[NPT];            // H weights
    bool valid[NPT];
};

// Sum of the production words at the first G source addresses (+ OFF bytes).
template <int G, uint32_t OFF>
__device__ __forceinline__ int pull_sum(const uint32_t (&src)[kInReg]) {
    int v[G];
#pragma unroll
    for (int e = 0; e < G; ++e) v[e] = lds_load(src[e] + OFF);
    int t = 0;
#pragma unroll
    for (int e = 0; e < G; ++e) t += v[e];
    return t;
}

// One step of the deterministic branch; prod is this step's production buffer
// (the even one, or the odd one kProdBytes further on when ODD).  Returns
// whether a neuron of this wave fired.  When no neuron of the block fires (a
// halting configuration) the step changes nothing, so halting is detected
// afterwards, once per batch of steps, from the waves' records.
template <int TPB, int NPT, bool ODD>
__device__ __forceinline__ bool det_step(Neurons<NPT>& N, const uint32_t* lrules, const uint32_t* lmagic, int* prod,
                                         const int* __restrict__ in_src, uint32_t count_max, bool& ovf) {
    constexpr uint32_t kOff = ODD ? 4u * (TPB * NPT + kZeros) : 0u;
    int fc[NPT];
    bool any = false;
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
        const int n = N.cnt[q];
        const bool small = n < N.S[q];
        const bool table = small || n >= N.T[q];
        // one lookup (the count itself below 16, else its residue mod 24):
        // entries 0-15 from a 64-bit pair (s1:s0 or l1:l0), residues 16-23
        // from l2; shifts and selects, no indexing and no branch
        const uint32_t r = small ? (uint32_t)n : (uint32_t)n % 24u;
        const u64 lo = small ? (((u64)N.s1[q] << 32) | N.s0[q]) : (((u64)N.l1[q] << 32) | N.l0[q]);
        const uint32_t sh = 4u * (r & 15u);
        const int idx = table ? (int)((r < 16 ? (uint32_t)(lo >> sh) : (N.l2[q] >> sh)) & 15u) : 0;
        // the fired rule's (c, p): rules 1-3 from a register word (idx 0: none),
        // later ones from LDS
        uint32_t cp = (uint32_t)(N.cpw[q] >> (16u * (uint32_t)min(idx, 3))) & 0xFFFFu;
        if (N.far[q] && __any(idx > 3)) {
            if (idx > 3) {
                const uint32_t R = lrules[N.rs[q] + idx - 1];
                cp = ((R >> 16) & 0xFFu) | ((R >> 24) << 8);
            }
        }
        bool found = idx != 0;
        if (N.slow[q] && __any(!table)) {
            // first applicable rule, over the wave's largest rule count (no early exit)
            for (int k = 0; k < N.rw[q]; ++k) {
                const int kk = N.rs[q] + min(k, max(N.rn[q] - 1, 0));
                const uint32_t R = lrules[kk];
                const bool ok = !table && !found && k < N.rn[q] && applies_packed(n, R, lmagic[kk]);
                cp = ok ? (((R >> 16) & 0xFFu) | ((R >> 24) << 8)) : cp;
                found |= ok;
            }
        }
        fc[q] = (int)(cp & 0xFFu);
        any |= found;
        prod[threadIdx.x + q * TPB] = (int)(cp >> 8);  // a slot past m writes 0 to its own word
    }
    const bool wave_fired = __any(any);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
        // unconditional reads, all issued before the first add (a lane past
        // its in-degree reads a zero word): 4, 8, ..., 32 of them by the wave's
        // largest in-degree (uniform; slots are ordered by in-degree, so a
        // wave's neurons are alike)
        const int kw = N.kw[q];
        int recv;
        if (kw > 16) {
            if (kw > 28) recv = pull_sum<32, kOff>(N.src[q]);
            else if (kw > 24) recv = pull_sum<28, kOff>(N.src[q]);
            else if (kw > 20) recv = pull_sum<24, kOff>(N.src[q]);
            else recv = pull_sum<20, kOff>(N.src[q]);
        } else {
            if (kw > 12) recv = pull_sum<16, kOff>(N.src[q]);
            else if (kw > 8) recv = pull_sum<12, kOff>(N.src[q]);
            else if (kw > 4) recv = pull_sum<8, kOff>(N.src[q]);
            else recv = pull_sum<4, kOff>(N.src[q]);
        }
        for (int e = kInReg; e < N.in[q]; ++e) recv += prod[in_src[N.is[q] + e]];
        // a fired rule consumes at most the count (c <= n), and recv < 2^21
        // (p <= 255, at most 4096 sources), so the new count fits 32 bits
        const uint32_t v = (uint32_t)N.cnt[q] - (uint32_t)fc[q] + (uint32_t)recv;
        ovf |= v > count_max;
        N.cnt[q] = (int)v;
    }
    return wave_fired;
}

// det_step with the parity known only at run time (re-simulations).
template <int TPB, int NPT>
__device__ __forceinline__ void det_step_any(Neurons<NPT>& N, int t, const uint32_t* lrules, const uint32_t* lmagic,
                                             int* prod0, int* prod1, const int* __restrict__ in_src,
                                             uint32_t count_max, bool& ovf) {
    if (t & 1) det_step<TPB, NPT, true>(N, lrules, lmagic, prod1, in_src, count_max, ovf);
    else det_step<TPB, NPT, false>(N, lrules, lmagic, prod0, in_src, count_max, ovf);
}

template <int NPT>
__device__ __forceinline__ u64 h_partial(const Neurons<NPT>& N) {
    u64 h = 0;
#pragma unroll
    for (int q = 0; q < NPT; ++q)
        h += (u64)(uint32_t)N.cnt[q] * N.R[q];  // R = 0 past m
    return h;
}

template <typename T, int TPB, int NPT>
__device__ __forceinline__ void load_counts(Neurons<NPT>& N, const T* row) {
#pragma unroll
    for (int q = 0; q < NPT; ++q)
        if (N.valid[q]) N.cnt[q] = (int)row[threadIdx.x + q * TPB];
}

template <typename T, int TPB, int NPT>
__device__ __forceinline__ void store_counts(const Neurons<NPT>& N, T* row) {
#pragma unroll
    for (int q = 0; q < NPT; ++q)
        if (N.valid[q]) row[threadIdx.x + q * TPB] = (T)N.cnt[q];
}

// The counts into a row of HBM, each at its neuron's place.
template <typename T, int TPB, int NPT>
__device__ __forceinline__ void store_final(const Neurons<NPT>& N, T* row) {
#pragma unroll
    for (int q = 0; q < NPT; ++q)
        if (N.valid[q]) row[N.orig[q]] = (T)N.cnt[q];
}

// Block-wide H of the current counts (every thread gets it).
template <int TPB, int NPT>
__device__ __forceinline__ u64 block_hash(const Neurons<NPT>& N, u64* bpart) {
    const u64 w = wave_sum64(h_partial(N));
    if ((threadIdx.x & 63) == 0) bpart[threadIdx.x >> 6] = w;
    __syncthreads();
    u64 h = 0;
    for (int q = 0; q < TPB / 64; ++q) h += bpart[q];
    __syncthreads();  // bpart may be rewritten afterwards
    return h;
}

struct BatchLds {
    int* prod0;        // [slots + kZeros] at the start of LDS; the last kZeros words always hold 0
    int* prod1;        // [slots + kZeros] right after prod0 (4 (slots + kZeros) bytes on)
    uint32_t* lrules;  // [r_max]
    uint32_t* lmagic;  // [r_max]
    int* xrow;         // [slots] a configuration under verification
    u64* wpart;        // [(kBatch + 1) * waves]: per-wave partial H of every step of the batch
    u64* bpart;        // [waves]
    u64* hring;        // [kBatch + 1]: H(C_{batch_start + i})
    u64* term;         // [kBatch + 1]: digest terms of the batch
    int* cand;         // [kBatch + 1]: earliest step with an equal H
    u64* fired;        // [waves]: steps of the batch where a neuron of the wave fired
};

// slots = TPB * NPT (a multiple of 32, so each production buffer is a whole
// number of 16-byte units, prod1 starts exactly 4 (slots + kZeros) bytes on,
// and zero word b sits in LDS bank b).
__host__ __device__ __forceinline__ size_t lds_layout(int slots, int r_max, int waves, unsigned char* base,
                                                      BatchLds* L) {
    const size_t r4 = ((size_t)r_max + 3) & ~(size_t)3;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        unsigned char* p = base ? base + o : nullptr;
        o += (bytes + 15) & ~(size_t)15;
        return p;
    };
    unsigned char* p_prod0 = take(((size_t)slots + kZeros) * 4);
    unsigned char* p_prod1 = take(((size_t)slots + kZeros) * 4);
    unsigned char* p_rules = take(r4 * 4);
    unsigned char* p_magic = take(r4 * 4);
    unsigned char* p_xrow = take((size_t)slots * 4);
    unsigned char* p_wpart = take((size_t)(kBatch + 1) * waves * 8);
    unsigned char* p_bpart = take((size_t)waves * 8);
    unsigned char* p_hring = take((kBatch + 1) * 8);
    unsigned char* p_term = take((kBatch + 1) * 8);
    unsigned char* p_cand = take((kBatch + 1) * 4);
    unsigned char* p_fired = take((size_t)waves * 8);
    if (L) {
        L->lrules = (uint32_t*)p_rules;
        L->lmagic = (uint32_t*)p_magic;
        L->prod0 = (int*)p_prod0;
        L->prod1 = (int*)p_prod1;
        L->xrow = (int*)p_xrow;
        L->wpart = (u64*)p_wpart;
        L->bpart = (u64*)p_bpart;
        L->hring = (u64*)p_hring;
        L->term = (u64*)p_term;
        L->cand = (int*)p_cand;
        L->fired = (u64*)p_fired;
    }
    return o;
}

}  // namespace

size_t batch_lds_bytes(int r_max, int threads, int npt) {
    return lds_layout(threads * npt, r_max, threads / 64, nullptr, nullptr);
}

int batch_max_threads() { return kMaxThreads; }
int batch_interval() { return kBatch; }

template <typename T, int TPB, int NPT>
__global__ __launch_bounds__(TPB) void k_batch_det(BatchArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int W = TPB / 64;
    const int sys = blockIdx.x;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const BatchSys B = a.sys[sys];
    BatchLds L;
    constexpr int kSlots = TPB * NPT;
    lds_layout(kSlots, a.r_max, W, smem, &L);

    for (int q = threadIdx.x; q < B.r; q += TPB) {
        L.lrules[q] = a.rules[B.rule_off + q];
        L.lmagic[q] = a.magic[B.rule_off + q];
    }
    if (threadIdx.x < kZeros) L.prod0[kSlots + threadIdx.x] = L.prod1[kSlots + threadIdx.x] = 0;  // zero words
    const uint32_t pbase = lds_addr(L.prod0);

    Neurons<NPT> N;
    const T* c0 = (const T*)a.c0 + B.row_off;
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
        const int j = threadIdx.x + q * TPB;
        N.valid[q] = j < B.m;
        N.cnt[q] = 0;
        N.T[q] = 0x7FFFFFFF;
        N.S[q] = N.valid[q] ? 0 : 16;  // a slot past m: no rule ever applies (its small table is 0)
        N.l0[q] = N.l1[q] = N.l2[q] = N.s0[q] = N.s1[q] = 0;
        N.cpw[q] = 0;
        N.orig[q] = 0;
        N.rs[q] = N.rn[q] = N.is[q] = N.in[q] = 0;
        N.R[q] = 0;
#pragma unroll
        for (int e = 0; e < kInReg; ++e) N.src[q][e] = pbase + 4u * kSlots;  // a zero word
        if (N.valid[q]) {
            const int o = a.perm[B.nrp_off + j];
            N.orig[q] = o;
            N.cnt[q] = (int)c0[o];
            N.rs[q] = a.nrp[B.nrp_off + j];
            N.rn[q] = a.nrp[B.nrp_off + j + 1] - N.rs[q];
            N.is[q] = B.in_off + a.in_ptr[B.nrp_off + j];
            N.in[q] = a.in_ptr[B.nrp_off + j + 1] - a.in_ptr[B.nrp_off + j];
            N.R[q] = mix64((u64)(o + 1) * kGamma);
            for (int k = 0; k < min(N.rn[q], 3); ++k) {
                const uint32_t R = a.rules[B.rule_off + N.rs[q] + k];
                N.cpw[q] |= (u64)(((R >> 16) & 0xFFu) | ((R >> 24) << 8)) << (16 * (k + 1));
            }
            const uint32_t f = a.fast[B.nrp_off + j];
            const uint32_t* lt = a.lut + 5 * (B.nrp_off + j);
            if (f >> 31) {
                N.T[q] = (int)(f & 0xFFFFu);
                N.l0[q] = lt[0];
                N.l1[q] = lt[1];
                N.l2[q] = lt[2];
            }
            if (f & 0x40000000u) {
                N.S[q] = 16;
                N.s0[q] = lt[3];
                N.s1[q] = lt[4];
            }
            const uint16_t* rg = a.reg_src + (B.row_off + j) * kInReg;
#pragma unroll
            for (int e = 0; e < kInReg; ++e) {
                const uint32_t v = rg[e];
                N.src[q][e] = pbase + 4u * (v >= 0xFFE0u ? (uint32_t)kSlots + (v & 31u) : v);
            }
        }
        int kw = min(N.in[q], kInReg), rw = N.rn[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            kw = max(kw, __shfl_xor(kw, o));
            rw = max(rw, __shfl_xor(rw, o));
        }
        N.kw[q] = __builtin_amdgcn_readfirstlane(kw);
        N.rw[q] = __builtin_amdgcn_readfirstlane(rw);
        // every count of a lane is covered by the tables when the small one
        // exists (S = 16) and the residue one starts by 16 (a slot past m: count 0)
        N.far[q] = __any(N.valid[q] && N.rn[q] > 3);
        N.slow[q] = __any(N.valid[q] && !(N.S[q] == 16 && N.T[q] <= 16));
    }
    T* ckpt = (T*)a.ckpt + a.ckpt_rows * B.row_off;  // row q = the configuration at step q * kBatch
    u64* hkey = a.hkey + (u64)sys * a.table_slots;
    int* hstep = a.hstep + (u64)sys * a.table_slots;  // -1: empty slot
    const u64 hmask = a.table_slots - 1;
    const int steps = a.steps;
    __syncthreads();

    store_counts<T, TPB, NPT>(N, ckpt);
    const u64 h0 = block_hash<TPB, NPT>(N, L.bpart);
    u64 digest = mix64(h0);  // meaningful in thread 0
    if (threadIdx.x == 0) L.hring[0] = h0;
    int k = 0, batch_start = 0, halt = -1, first_rep = -1;
    bool ovf = false, collision = false;
    const uint32_t cmax = (uint32_t)a.count_max;

    for (;;) {
        // the batch's steps (batch_start is a multiple of kBatch: step
        // batch_start + i reads buffer i & 1), in groups of kGroup
        const int nb_run = min(kBatch, steps - batch_start);
        u64 fired = 0;  // bit i: a neuron of this wave fired at the step from C_{batch_start + i}
        for (int i = 0; i < nb_run; i += kGroup) {
            u64 hv[kGroup];
#pragma unroll
            for (int u = 0; u < kGroup; ++u) {
                hv[u] = 0;
                if (i + u < nb_run) {
                    const bool wf = (u & 1)
                        ? det_step<TPB, NPT, true>(N, L.lrules, L.lmagic, L.prod1, a.in_src, cmax, ovf)
                        : det_step<TPB, NPT, false>(N, L.lrules, L.lmagic, L.prod0, a.in_src, cmax, ovf);
                    fired |= (wf ? 1ULL : 0ULL) << (i + u);
                    hv[u] = h_partial(N);
                }
            }
            const u64 hs = wave_sum4(hv, lane);  // the wave's part of H(C_{batch_start + i + (lane & 3) + 1})
            if (lane < kGroup && i + lane < nb_run) L.wpart[(i + lane + 1) * W + wid] = hs;
        }
        k = batch_start + nb_run;
        bool done = k >= steps;

        // ---- batch boundary (or end of run) ----
        int nb = k - batch_start;  // H(C_{batch_start + i}) in hring[i], i = 0 .. nb
        // the first configuration of the batch where no neuron fired is halting;
        // the steps computed after it changed nothing
        if (lane == 0) L.fired[wid] = fired;
        __syncthreads();
        {
            u64 fm = 0;
            for (int w = 0; w < W; ++w) fm |= L.fired[w];
            const u64 stepped = nb >= 64 ? ~0ULL : ((1ULL << nb) - 1);
            const u64 idle = ~fm & stepped;
            if (idle) {
                nb = __builtin_ctzll(idle);
                k = batch_start + nb;
                halt = k;
                done = true;
            }
        }
        if (done) store_final<T, TPB, NPT>(N, (T*)a.final_out + B.row_off);
        if (k - batch_start == kBatch)  // a whole batch: the checkpoint of step k
            store_counts<T, TPB, NPT>(N, ckpt + (long long)(k / kBatch) * B.m);
        __syncthreads();  // the batch's per-wave partials are complete
        {
            const int i = threadIdx.x;
            if (i >= 1 && i <= nb) {
                u64 h = 0;
                for (int w = 0; w < W; ++w) h += L.wpart[i * W + w];
                L.hring[i] = h;
                L.term[i] = mix64(h + (u64)(batch_start + i) * kGamma);
            }
        }
        __syncthreads();
        if (wid == 0) {
            const u64 s = wave_sum64(lane < nb ? L.term[lane + 1] : 0);
            if (lane == 0) digest += s;
        }
        bool resimulated = false;
        if (first_rep < 0 && a.detect_repeats) {
            const int first_new = (batch_start == 0) ? 0 : 1;  // H(C_batch_start) is already in the set
            const int i = threadIdx.x;
            if (i <= kBatch) L.cand[i] = -1;
            __syncthreads();
            if (i >= first_new && i <= nb) {  // earlier batches: read-only probes
                const u64 key = L.hring[i];
                u64 s = (key * kGamma) >> 17;
                for (u64 it = 0; it <= hmask; ++it, ++s) {
                    const int st = hstep[s & hmask];
                    if (st < 0) break;
                    if (hkey[s & hmask] == key) {
                        L.cand[i] = st;
                        break;
                    }
                }
                if (L.cand[i] < 0)  // within this batch
                    for (int l = 0; l < i; ++l)
                        if (L.hring[l] == key) {
                            L.cand[i] = batch_start + l;
                            break;
                        }
            }
            __syncthreads();
            // confirm candidates in step order by re-simulating both rows
            for (int q = first_new; q <= nb && first_rep < 0; ++q) {
                const int l = L.cand[q];
                if (l < 0) continue;
                const int kk = batch_start + q;
                resimulated = true;
                load_counts<T, TPB, NPT>(N, ckpt + (long long)(l / kBatch) * B.m);
                for (int t = (l / kBatch) * kBatch; t < l; ++t)
                    det_step_any<TPB, NPT>(N, t, L.lrules, L.lmagic, L.prod0, L.prod1, a.in_src, cmax, ovf);
                store_counts<int, TPB, NPT>(N, L.xrow);
                load_counts<T, TPB, NPT>(N, ckpt + (long long)(kk / kBatch) * B.m);
                for (int t = (kk / kBatch) * kBatch; t < kk; ++t)
                    det_step_any<TPB, NPT>(N, t, L.lrules, L.lmagic, L.prod0, L.prod1, a.in_src, cmax, ovf);
                bool diff = false;
#pragma unroll
                for (int u = 0; u < NPT; ++u)
                    if (N.valid[u]) diff |= (L.xrow[threadIdx.x + u * TPB] != N.cnt[u]);
                if (__syncthreads_or(diff) == 0) first_rep = kk;
                else collision = true;
            }
            // insert the first occurrence of every new H value
            if (i >= first_new && i <= nb && L.cand[i] < 0) {
                const u64 key = L.hring[i];
                u64 s = (key * kGamma) >> 17;
                for (u64 it = 0; it <= hmask; ++it, ++s)
                    if (atomicCAS(&hstep[s & hmask], -1, batch_start + i) == -1) {
                        hkey[s & hmask] = key;
                        break;
                    }
            }
            __syncthreads();
        }
        if (done) break;
        if (resimulated)  // back to the configuration at step k
            load_counts<T, TPB, NPT>(N, ckpt + (long long)(k / kBatch) * B.m);
        if (threadIdx.x == 0) L.hring[0] = L.hring[nb];
        batch_start = k;
        __syncthreads();
    }
    const bool any_ovf = __syncthreads_or(ovf) != 0;
    const bool any_col = __syncthreads_or(collision) != 0;
    if (threadIdx.x == 0) {
        a.halt_step[sys] = halt;
        a.first_repeat[sys] = first_rep;
        a.steps_done[sys] = k;
        a.digest[sys] = digest;
        a.err[sys] = (any_ovf ? 1ULL : 0ULL) | (any_col ? 2ULL : 0ULL);
    }
}

hipError_t launch_batch_det(int elem_bytes, int threads, int npt, const BatchArgs& a, int n_sys, hipStream_t st) {
    if (n_sys <= 0) return hipSuccess;
    const size_t lds = batch_lds_bytes(a.r_max, threads, npt);
#define SNP_BATCH(TT, TPB, NN) \
    hipLaunchKernelGGL((k_batch_det<TT, TPB, NN>), dim3(n_sys), dim3(TPB), lds, st, a)
#define SNP_BATCH_NPT(TT, TPB)                      \
    do {                                            \
        if (npt == 1) SNP_BATCH(TT, TPB, 1);        \
        else if (npt == 2) SNP_BATCH(TT, TPB, 2);   \
        else SNP_BATCH(TT, TPB, 4);                 \
    } while (0)
#define SNP_BATCH_TPB(TT)                                  \
    do {                                                   \
        if (threads == 256) SNP_BATCH_NPT(TT, 256);        \
        else if (threads == 512) SNP_BATCH_NPT(TT, 512);   \
        else SNP_BATCH_NPT(TT, 1024);                      \
    } while (0)
    if (!((threads == 256 || threads == 512 || threads == 1024) && (npt == 1 || npt == 2 || npt == 4)))
        return hipErrorInvalidValue;
    if (elem_bytes == 4) SNP_BATCH_TPB(int32_t);
    else SNP_BATCH_TPB(uint16_t);
#undef SNP_BATCH_TPB
#undef SNP_BATCH_NPT
#undef SNP_BATCH
    return hipGetLastError();
}

}  // namespace snp
