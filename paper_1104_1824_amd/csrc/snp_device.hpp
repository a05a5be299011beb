// Device helpers shared by the kernels of libsnp (gfx950, wave64).
#pragma once

#include "snp_internal.hpp"

namespace snp {

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ u64 sat_mul(u64 a, u64 b) {
    if (a == 0 || b == 0) return 0;
    if (a >= kPsiSat || b >= kPsiSat) return kPsiSat;
    const u64 hi = __umul64hi(a, b);
    const u64 lo = a * b;
    return (hi != 0 || lo >= kPsiSat) ? kPsiSat : lo;
}

__device__ __forceinline__ u64 sat_add(u64 a, u64 b) {  // a, b <= 2^62: no wrap
    const u64 s = a + b;
    return s >= kPsiSat ? kPsiSat : s;
}

__device__ __forceinline__ u64 uni64(u64 x) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((u64)hi << 32) | lo;
}

__device__ __forceinline__ long long uni_ll(long long x) { return (long long)uni64((u64)x); }

// Orders this wave's LDS traffic: LDS operations of one wavefront complete in
// issue order, so a compiler-level fence plus a wave barrier is enough for
// lanes to see each other's writes.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Wave64 reductions on DPP: inclusive sums within rows of 16 lanes by row
// shifts 1, 2, 4, 8 (lanes shifted in from outside the row read 0), then
// row broadcasts of lanes 15 and 31 carry the row totals upward; lane 63 ends
// with the total, which is returned to every lane.  All 64 lanes must be
// active.
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    v += __builtin_amdgcn_update_dpp(0u, v, 0x111, 0xf, 0xf, true);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0u, v, 0x112, 0xf, 0xf, true);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0u, v, 0x114, 0xf, 0xf, true);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0u, v, 0x118, 0xf, 0xf, true);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0u, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0u, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

// Maximum of non-negative values (0 is the identity).
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0x111, 0xf, 0xf, true));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0x112, 0xf, 0xf, true));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0x114, 0xf, 0xf, true));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0x118, 0xf, 0xf, true));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0x142, 0xa, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0u, v, 0x143, 0xc, 0xf, false));
    return __builtin_amdgcn_readlane(v, 63);
}

// 64-bit wave sum (mod 2^64) on the same DPP pattern, carries included.
#define SNP_DPP_ADD64(V, CTRL, RM, BC)                                                              \
    do {                                                                                            \
        const uint32_t lo_ = __builtin_amdgcn_update_dpp(0u, (uint32_t)(V), CTRL, RM, 0xf, BC);      \
        const uint32_t hi_ = __builtin_amdgcn_update_dpp(0u, (uint32_t)((V) >> 32), CTRL, RM, 0xf, BC); \
        (V) += ((u64)hi_ << 32) | lo_;                                                              \
    } while (0)

__device__ __forceinline__ u64 wave_sum_u64(u64 v) {
    SNP_DPP_ADD64(v, 0x111, 0xf, true);
    SNP_DPP_ADD64(v, 0x112, 0xf, true);
    SNP_DPP_ADD64(v, 0x114, 0xf, true);
    SNP_DPP_ADD64(v, 0x118, 0xf, true);
    SNP_DPP_ADD64(v, 0x142, 0xa, false);
    SNP_DPP_ADD64(v, 0x143, 0xc, false);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, 63);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), 63);
    return ((u64)hi << 32) | lo;
}

__device__ __forceinline__ int wave_max_i32(int x) { return (int)wave_max_u32((uint32_t)(x + 1)) - 1; }

// Inclusive prefix sums over the lanes (lane i: lanes 0 .. i), the partial
// results of the same DPP pattern; all 64 lanes active.
__device__ __forceinline__ uint32_t wave_incl_u32(uint32_t v) {
    v += __builtin_amdgcn_update_dpp(0u, v, 0x111, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x112, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x114, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x118, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x142, 0xa, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x143, 0xc, 0xf, false);
    return v;
}

__device__ __forceinline__ u64 wave_incl_u64(u64 v) {
    SNP_DPP_ADD64(v, 0x111, 0xf, true);
    SNP_DPP_ADD64(v, 0x112, 0xf, true);
    SNP_DPP_ADD64(v, 0x114, 0xf, true);
    SNP_DPP_ADD64(v, 0x118, 0xf, true);
    SNP_DPP_ADD64(v, 0x142, 0xa, false);
    SNP_DPP_ADD64(v, 0x143, 0xc, false);
    return v;
}

__device__ __forceinline__ uint32_t sat_mul32(uint32_t a, uint32_t b) {  // a, b >= 1
    return __umulhi(a, b) ? 0xFFFFFFFFu : a * b;
}

// Product over the lanes after this one (lane i: lanes i+1 .. 63, 1 for lane
// 63) of factors >= 1, saturated at 2^32 - 1: products along each row of 16
// by DPP row shifts toward lower lanes (lanes past the row's end read 1), the
// row products of later rows multiplied in from scalars, then a wave shift by
// one lane.  All 64 lanes active.
__device__ __forceinline__ uint32_t wave_after_prod_sat32(uint32_t v) {
    v = sat_mul32(v, (uint32_t)__builtin_amdgcn_update_dpp(1u, v, 0x101, 0xf, 0xf, false));  // row_shl:1
    v = sat_mul32(v, (uint32_t)__builtin_amdgcn_update_dpp(1u, v, 0x102, 0xf, 0xf, false));  // row_shl:2
    v = sat_mul32(v, (uint32_t)__builtin_amdgcn_update_dpp(1u, v, 0x104, 0xf, 0xf, false));  // row_shl:4
    v = sat_mul32(v, (uint32_t)__builtin_amdgcn_update_dpp(1u, v, 0x108, 0xf, 0xf, false));  // row_shl:8
    const uint32_t r1 = __builtin_amdgcn_readlane(v, 16), r2 = __builtin_amdgcn_readlane(v, 32);
    const uint32_t r3 = __builtin_amdgcn_readlane(v, 48);
    const uint32_t p23 = sat_mul32(r2, r3), p123 = sat_mul32(r1, p23);
    const int row = (int)(__lane_id() >> 4);
    v = sat_mul32(v, row == 0 ? p123 : row == 1 ? p23 : row == 2 ? r3 : 1u);
    return (uint32_t)__builtin_amdgcn_update_dpp(1u, v, 0x130, 0xf, 0xf, false);  // wave_shl:1
}

// Rule applicability: a^n in L(a^i (a^j)*) and n >= c.
__device__ __forceinline__ bool rule_applies(int n, const int4 R) {
    if (n < R.x || n < R.z) return false;
    if (R.y == 0) return n == R.x;
    return ((n - R.x) % R.y) == 0;
}

// Index of the d-th set bit of mask (d < popcount(mask)).
__device__ __forceinline__ int nth_bit(uint32_t mask, int d) {
    for (int q = 0; q < d; ++q) mask &= mask - 1;
    return __ffs(mask) - 1;
}

// Configuration hash.  H(C) = sum over neurons n of C[n] * R[n] (mod 2^64),
// R[n] = mix64((n + 1) * gamma) (the SplitMix64 stream), which is linear in C:
// H(C + M_k) = H(C) + H(M_k) for a row M_k of M_Pi.  The visited-set key is
// fmix64(H) (MurmurHash3's 64-bit finaliser), masked by the hash_mask option.
__device__ __forceinline__ u64 fmix64(u64 k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

__device__ __forceinline__ u64 hterm(uint32_t v, u64 R) { return (u64)v * R; }

template <typename T>
__device__ __forceinline__ u64 row_hash_wave(const T* row, const u64* R, int m, int lane) {
    u64 h = 0;
    for (int j = lane; j < m; j += 64) h += hterm((uint32_t)row[j], R[j]);
    return wave_sum_u64(h);
}

// Twin rules: two rules of one neuron with the same consumption c and the same
// production p have identical rows of M_Pi (Definition 2), so a child that
// fires the later one of two applicable twins equals the child that fires the
// earlier one with every other choice unchanged, which has a smaller index t:
// it is never a first occurrence.  Digit d of a neuron is "canonical" when no
// earlier applicable rule of the neuron is its twin.
__device__ __forceinline__ uint32_t canonical_mask(const int4* rules, int r0, uint32_t app) {
    uint32_t cm = 0;
    int d = 0;
    for (uint32_t a = app; a; a &= a - 1, ++d) {
        const int q = __ffs(a) - 1;
        const int4 R = rules[r0 + q];
        bool canon = true;
        for (uint32_t b = app & ((1u << q) - 1); b; b &= b - 1) {
            const int4 Q = rules[r0 + __ffs(b) - 1];
            if (Q.z == R.z && Q.w == R.w) {
                canon = false;
                break;
            }
        }
        cm |= canon ? (1u << d) : 0u;
    }
    return cm;
}

// Canonical enumeration.  A child is computed only when every neuron's digit
// is canonical (twins never are: they repeat an earlier child); canonical
// children are numbered u = 0, 1, ... in the same order as their child
// indices t (Algorithm 2 II-3 order restricted to them), as a mixed-radix
// number whose digit e of a neuron counts the canonical digits below its
// digit.  kappa = number of canonical digits of a neuron (1 when omega <= 1:
// its only value fires its one rule, or nothing).  am holds the applicable
// rules in its low 16 bits and, for omega >= 2, the canonical digits above.
__device__ __forceinline__ int kappa_of(uint32_t am, int om) { return om >= 2 ? __popc(am >> 16) : 1; }

// Digit (ordinal among the applicable rules) of canonical digit e.
__device__ __forceinline__ int canon_digit(uint32_t am, int om, int e) { return om >= 2 ? nth_bit(am >> 16, e) : 0; }

// Saturating sum over the wave (values <= 2^62).
__device__ __forceinline__ u64 wave_satsum(u64 x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = sat_add(x, __shfl_xor(x, o));
    return x;
}

// Applicable-rule mask of a neuron holding x spikes (rules r0 .. r1 - 1) with
// its canonical digits in the high 16 bits (omega >= 2), and omega.
__device__ __forceinline__ uint32_t neuron_applicable(int x, int r0, int r1, const int4* rules, int& w) {
    uint32_t mask = 0;
    w = 0;
    for (int q = r0; q < r1; ++q)
        if (rule_applies(x, rules[q])) {
            mask |= 1u << (q - r0);
            ++w;
        }
    return mask | (w >= 2 ? canonical_mask(rules, r0, mask) << 16 : 0xFFFF0000u);
}

// With delays: the steps neuron j (< mcount) still waits before it sends its
// delayed spikes (0: open).  dlink[j] is the column of its wait entry in a row
// (-1: the neuron owns no rule with a delay); dlink null: a system without
// delays.
template <typename T>
__device__ __forceinline__ int neuron_wait(const T* row, const int* dlink, int mcount, int j) {
    if (!dlink || j >= mcount) return 0;
    const int c = dlink[j];
    return c >= 0 ? (int)row[c] : 0;
}

// Mixed-radix decode of child index t (Algorithm 2 II-3 order: the last neuron
// is the least significant digit; a neuron with omega <= 1 has one value).
// Lane L owns the contiguous neurons [L*Q, L*Q + Q); the place value of its
// block is a suffix product across lanes (saturated at 2^62, above any t),
// which depends on the parent only (digit_place) and can be kept across
// decodes of children of one parent (decode_digits_at).
__device__ __forceinline__ u64 digit_place(int m, int lane, const uint8_t* om) {
    const int Q = (m + 63) >> 6;
    const int j0 = lane * Q;
    const int j1 = min(m, j0 + Q);
    u64 bp = 1;
    for (int j = j0; j < j1; ++j) bp = sat_mul(bp, (u64)max(1, (int)om[j]));
    u64 incl = bp;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const u64 y = __shfl_down(incl, o);
        if (lane + o < 64) incl = sat_mul(incl, y);
    }
    u64 after = __shfl_down(incl, 1);
    if (lane == 63) after = 1;
    return after;
}

__device__ __forceinline__ void decode_digits_at(int m, int lane, u64 t, const uint8_t* om, uint8_t* dg, u64 after) {
    const int Q = (m + 63) >> 6;
    const int j0 = lane * Q;
    const int j1 = min(m, j0 + Q);
    u64 tl = (after > t) ? 0 : t / after;
    if (tl == 0) {  // every digit of this lane's neurons is 0 (the usual case far from the end)
        for (int j = j0; j < j1; ++j) dg[j] = 0;
    } else if (tl <= 0xFFFFFFFFull) {  // 32-bit divisions suffice
        uint32_t t32 = (uint32_t)tl;
        for (int j = j1 - 1; j >= j0; --j) {
            const uint32_t w = (uint32_t)max(1, (int)om[j]);
            const uint32_t q = t32 / w;
            dg[j] = (uint8_t)(t32 - q * w);
            t32 = q;
        }
    } else {
        for (int j = j1 - 1; j >= j0; --j) {
            const uint32_t w = (uint32_t)max(1, (int)om[j]);
            dg[j] = (uint8_t)(tl % w);
            tl /= w;
        }
    }
}

__device__ __forceinline__ void decode_digits(int m, int lane, u64 t, const uint8_t* om, uint8_t* dg) {
    decode_digits_at(m, lane, t, om, dg, digit_place(m, lane, om));
}

// Place values of the canonical digits (product of kappa over the later
// neurons) and canonical decode, for the lane's block of neurons as in
// digit_place / decode_digits_at.
__device__ __forceinline__ u64 canon_place(int m, int lane, const uint8_t* om, const uint32_t* am) {
    const int Q = (m + 63) >> 6;
    const int j0 = lane * Q;
    const int j1 = min(m, j0 + Q);
    u64 bp = 1;
    for (int j = j0; j < j1; ++j) bp = sat_mul(bp, (u64)kappa_of(am[j], om[j]));
    u64 incl = bp;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const u64 y = __shfl_down(incl, o);
        if (lane + o < 64) incl = sat_mul(incl, y);
    }
    u64 after = __shfl_down(incl, 1);
    if (lane == 63) after = 1;
    return after;
}

__device__ __forceinline__ void canon_decode(int m, int lane, u64 u, const uint8_t* om, const uint32_t* am,
                                             uint8_t* eg, u64 after) {
    const int Q = (m + 63) >> 6;
    const int j0 = lane * Q;
    const int j1 = min(m, j0 + Q);
    u64 tl = (after > u) ? 0 : u / after;
    for (int j = j1 - 1; j >= j0; --j) {
        if (tl == 0) {
            eg[j] = 0;
            continue;
        }
        const uint32_t k = (uint32_t)kappa_of(am[j], om[j]);
        eg[j] = (uint8_t)(tl % k);
        tl /= k;
    }
}

// Child index t of a canonical child whose canonical digits are eg: the sum
// over neurons of digit * (product of max(1, omega) over the later neurons),
// lane L summing its block [L*Q, L*Q + Q) and scaling by the block's place
// value after_w (digit_place over omega).  Arithmetic is mod 2^64; it is exact
// because every enumerated child has t < 2^62 (a saturated place value then
// only ever meets digit 0).  All 64 lanes active; every lane gets t.
__device__ __forceinline__ u64 child_index(int m, int lane, const uint8_t* om, const uint32_t* am, const uint8_t* eg,
                                           u64 after_w) {
    const int Q = (m + 63) >> 6;
    const int j0 = lane * Q;
    const int j1 = min(m, j0 + Q);
    u64 v = 0, pl = 1;
    for (int j = j1 - 1; j >= j0; --j) {
        const int w = om[j];
        if (w >= 2) {
            v += (u64)canon_digit(am[j], w, eg[j]) * pl;
            pl *= (u64)w;
        }
    }
    return wave_sum_u64(v * after_w);
}

}  // namespace snp
