// gfx950 kernels of the breadth-first expansion of an SN P system's computation
// tree.  One level is: applicability and child counts Psi per parent, an
// exclusive prefix sum of Psi, then chunks of consecutive children g that are
// decoded (mixed radix), computed as C' = C + S.M (Equation next-config),
// hashed, deduplicated against the visited set and committed in order.
//
// Wave64 throughout: one wavefront per parent (Psi), per run of consecutive
// children (expand), or per child (insert / commit), lanes striding over the
// neurons of a row so that row loads and stores are contiguous.
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

__device__ __forceinline__ u64 wave_sum_u64(u64 x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

__device__ __forceinline__ int wave_max_i32(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o));
    return x;
}

__device__ __forceinline__ u64 wave_satprod(u64 x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = sat_mul(x, __shfl_xor(x, o));
    return x;
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

// Configuration hash: sum over neurons of a 64-bit finaliser (MurmurHash3
// fmix64) of (neuron, count).  Order independent across lanes, position
// dependent through the neuron index.
__device__ __forceinline__ u64 fmix64(u64 k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

__device__ __forceinline__ u64 elem_hash(int j, uint32_t v) {
    return fmix64((((u64)(uint32_t)j << 32) | v) ^ 0x9E3779B97F4A7C15ULL);
}

template <typename T>
__device__ __forceinline__ u64 row_hash_wave(const T* row, int m, int lane) {
    u64 h = 0;
    for (int j = lane; j < m; j += 64) h += elem_hash(j, (uint32_t)row[j]);
    return wave_sum_u64(h);
}

// ---------------------------------------------------------------------------
// Psi: per parent, number of valid spiking vectors (Algorithm 2 II-1/II-2):
// product over neurons of max(1, omega_n), saturated; 0 when no rule applies
// anywhere (halting) or when the parent exceeds the expansion count limit.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_psi(DevSystem s, const T* __restrict__ F, long long n,
                                             long long expand_max, u64* __restrict__ psi,
                                             DevCounters* __restrict__ ctr) {
    const int lane = threadIdx.x & 63;
    const long long p = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (p >= n) return;
    const T* row = F + p * (long long)s.m;
    u64 prod = 1;
    bool any = false, over = false;
    for (int j = lane; j < s.m; j += 64) {
        const int x = (int)row[j];
        int w = 0;
        const int r1 = s.nrule_ptr[j + 1];
        for (int q = s.nrule_ptr[j]; q < r1; ++q) w += rule_applies(x, s.rules[q]) ? 1 : 0;
        any |= (w > 0);
        over |= (expand_max >= 0 && (long long)x > expand_max);
        prod = sat_mul(prod, (u64)(w > 1 ? w : 1));
    }
    prod = wave_satprod(prod);
    const bool wany = __any(any);
    const bool wover = __any(over);
    if (lane == 0) {
        psi[p] = (!wany || wover) ? 0 : prod;
        if (!wany) atomicAdd(&ctr->halting, 1ULL);
    }
}

hipError_t launch_psi(int elem_bytes, const DevSystem& s, const void* frontier, long long n,
                      long long expand_max, u64* psi, DevCounters* ctr, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n + 3) / 4);
    if (elem_bytes == 4)
        hipLaunchKernelGGL(k_psi<int32_t>, dim3(blocks), dim3(256), 0, st, s, (const int32_t*)frontier, n,
                           expand_max, psi, ctr);
    else
        hipLaunchKernelGGL(k_psi<uint16_t>, dim3(blocks), dim3(256), 0, st, s, (const uint16_t*)frontier, n,
                           expand_max, psi, ctr);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exclusive prefix sums (tiles of 1024 = 256 threads x 4; wave64 shuffles, then
// the four wave totals through LDS; tile totals scanned by one block).
// ---------------------------------------------------------------------------
template <typename V, bool SAT>
__device__ __forceinline__ V vadd(V a, V b) {
    if constexpr (SAT) return (V)sat_add((u64)a, (u64)b);
    else return a + b;
}

constexpr int kScanTile = 1024;

template <typename V, bool SAT>
__global__ __launch_bounds__(256) void k_scan_tiles(const V* __restrict__ in, V* __restrict__ out,
                                                    V* __restrict__ tile_sums, long long n) {
    __shared__ V wsum[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const long long base = (long long)blockIdx.x * kScanTile + threadIdx.x * 4;
    V x[4], loc[4];
    V run = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        x[i] = (base + i < n) ? in[base + i] : (V)0;
        loc[i] = run;
        run = vadd<V, SAT>(run, x[i]);
    }
    V incl = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const V y = __shfl_up(incl, o);
        if (lane >= o) incl = vadd<V, SAT>(incl, y);
    }
    V excl = __shfl_up(incl, 1);
    if (lane == 0) excl = 0;
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    V wpre = 0;
    for (int w = 0; w < wid; ++w) wpre = vadd<V, SAT>(wpre, wsum[w]);
    const V tpre = vadd<V, SAT>(wpre, excl);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (base + i < n) out[base + i] = vadd<V, SAT>(tpre, loc[i]);
    if (threadIdx.x == 255) tile_sums[blockIdx.x] = vadd<V, SAT>(wpre, incl);
}

template <typename V, bool SAT>
__global__ __launch_bounds__(1024) void k_scan_sums(const V* __restrict__ sums, V* __restrict__ pre,
                                                    long long ntiles, u64* __restrict__ total) {
    __shared__ V wsum[16];
    __shared__ V carry_s;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (long long b = 0; b < ntiles; b += 1024) {
        const long long i = b + threadIdx.x;
        const V x = (i < ntiles) ? sums[i] : (V)0;
        V incl = x;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const V y = __shfl_up(incl, o);
            if (lane >= o) incl = vadd<V, SAT>(incl, y);
        }
        V excl = __shfl_up(incl, 1);
        if (lane == 0) excl = 0;
        if (lane == 63) wsum[wid] = incl;
        __syncthreads();
        V wpre = carry_s;
        for (int w = 0; w < wid; ++w) wpre = vadd<V, SAT>(wpre, wsum[w]);
        if (i < ntiles) pre[i] = vadd<V, SAT>(wpre, excl);
        __syncthreads();
        if (threadIdx.x == 1023) carry_s = vadd<V, SAT>(wpre, incl);
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = (u64)carry_s;
}

template <typename V, bool SAT>
__global__ __launch_bounds__(256) void k_scan_add(V* __restrict__ out, const V* __restrict__ pre, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = vadd<V, SAT>(pre[i / kScanTile], out[i]);
}

long long scan_tiles(long long n) { return (n + kScanTile - 1) / kScanTile; }

template <typename V, bool SAT>
static hipError_t scan_impl(const V* in, V* out, long long n, V* tile_sums, V* tile_pre, u64* total,
                            hipStream_t st) {
    const long long nt = scan_tiles(n);
    if (nt > 0) hipLaunchKernelGGL((k_scan_tiles<V, SAT>), dim3((unsigned)nt), dim3(256), 0, st, in, out, tile_sums, n);
    hipLaunchKernelGGL((k_scan_sums<V, SAT>), dim3(1), dim3(1024), 0, st, tile_sums, tile_pre, nt, total);
    if (nt > 1)
        hipLaunchKernelGGL((k_scan_add<V, SAT>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, out, tile_pre, n);
    return hipGetLastError();
}

hipError_t launch_scan_u64(const u64* in, u64* out, long long n, u64* tile_sums, u64* tile_pre, u64* total,
                           hipStream_t st) {
    return scan_impl<u64, true>(in, out, n, tile_sums, tile_pre, total, st);
}

hipError_t launch_scan_u32(const uint32_t* in, uint32_t* out, long long n, uint32_t* tile_sums,
                           uint32_t* tile_pre, u64* total, hipStream_t st) {
    return scan_impl<uint32_t, false>(in, out, n, tile_sums, tile_pre, total, st);
}

// ---------------------------------------------------------------------------
// Expansion, sparse form.  Every wave owns a run of consecutive children
// g0 + b0 .. g0 + b0 + run - 1.  Per wave, LDS holds the parent row, the
// applicable-rule mask and count omega of every neuron, the current digit of
// every neuron and the production p of every neuron's fired rule.
//
//   decode (once per run): place value of each lane's block of neurons is a
//     suffix product across lanes; digits follow by division.
//   advance (per child): add one to the mixed-radix number: the last neuron
//     with omega >= 2 whose digit is below omega - 1 steps up and every later
//     neuron with omega >= 2 resets to 0; past the last child of a parent the
//     wave moves to the next parent with Psi > 0, digits all 0.
//   child (per child): C'[d] = C[d] - c(fired rule of d) + sum over in-synapses
//     (s, d) of p(fired rule of s): the nonzero entries of column d of S.M.
// ---------------------------------------------------------------------------
constexpr int kLdsBytesPerNeuron = 4 /*par*/ + 4 /*prod*/ + 4 /*mask*/ + 1 /*omega*/ + 1 /*digit*/;

template <typename T>
__device__ __forceinline__ void load_parent(const DevSystem& s, const T* row, int lane, int* par, uint32_t* am,
                                            uint8_t* om) {
    for (int j = lane; j < s.m; j += 64) {
        const int x = (int)row[j];
        par[j] = x;
        uint32_t mask = 0;
        int w = 0;
        const int r0 = s.nrule_ptr[j], r1 = s.nrule_ptr[j + 1];
        for (int q = r0; q < r1; ++q)
            if (rule_applies(x, s.rules[q])) {
                mask |= 1u << (q - r0);
                ++w;
            }
        am[j] = mask;
        om[j] = (uint8_t)w;
    }
}

__device__ __forceinline__ void decode_digits(int m, int lane, u64 t, const uint8_t* om, uint8_t* dg) {
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
    u64 tl = (after > t) ? 0 : t / after;
    for (int j = j1 - 1; j >= j0; --j) {
        const uint32_t w = (uint32_t)max(1, (int)om[j]);
        dg[j] = (uint8_t)(tl % w);
        tl /= w;
    }
}

__device__ __forceinline__ void advance_digits(int m, int lane, const uint8_t* om, uint8_t* dg) {
    int myJ = -1;
    for (int j = lane; j < m; j += 64) {
        const int w = om[j];
        if (w >= 2 && dg[j] < w - 1) myJ = j;
    }
    const int J = wave_max_i32(myJ);
    for (int j = lane; j < m; j += 64) {
        const int w = om[j];
        if (j == J) dg[j] = (uint8_t)(dg[j] + 1);
        else if (w >= 2 && j > J) dg[j] = 0;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_expand_sparse(DevSystem s, ChunkArgs a, int run, int lds_stride) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const long long wave = (long long)blockIdx.x * (blockDim.x >> 6) + wid;
    const long long b0 = wave * run;
    if (b0 >= a.B) return;
    const int m = s.m;
    unsigned char* base = smem + (size_t)wid * lds_stride;
    int* par = (int*)base;
    int* prod = par + m;
    uint32_t* am = (uint32_t*)(prod + m);
    uint8_t* om = (uint8_t*)(am + m);
    uint8_t* dg = om + m;
    const T* F = (const T*)a.frontier;
    T* stage = (T*)a.stage;
    const int cnt = (int)min((long long)run, a.B - b0);

    // parent of the first child: last p with off[p] <= g (it has Psi > 0)
    const u64 g = a.g0 + (u64)b0;
    long long lo = 0, hi = a.n;
    while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if (a.off[mid] <= g) lo = mid + 1;
        else hi = mid;
    }
    long long p = uni_ll(lo - 1);
    u64 t = uni64(g - a.off[p]);
    u64 psi_p = uni64(a.psi[p]);
    load_parent<T>(s, F + p * (long long)m, lane, par, am, om);
    wave_lds_sync();
    decode_digits(m, lane, t, om, dg);
    wave_lds_sync();

    bool ovf = false;
    for (int k = 0; k < cnt; ++k) {
        const long long b = b0 + k;
        for (int j = lane; j < m; j += 64) {
            int pv = 0;
            if (om[j]) pv = s.rules[s.nrule_ptr[j] + nth_bit(am[j], dg[j])].w;
            prod[j] = pv;
        }
        wave_lds_sync();
        u64 h = 0;
        T* out = stage + b * (long long)m;
        for (int j = lane; j < m; j += 64) {
            long long v = par[j];
            if (om[j]) v -= s.rules[s.nrule_ptr[j] + nth_bit(am[j], dg[j])].z;
            const int e1 = s.in_ptr[j + 1];
            for (int e = s.in_ptr[j]; e < e1; ++e) v += prod[s.in_src[e]];
            ovf |= (v < 0) | (v > s.count_max);
            out[j] = (T)v;
            h += elem_hash(j, (uint32_t)v);
        }
        h = wave_sum_u64(h);
        if (lane == 0) {
            a.hash[b] = h & a.hash_mask;
            a.cpar[b] = (int)p;
            a.ct[b] = t;
        }
        wave_lds_sync();
        if (k + 1 < cnt) {
            ++t;
            if (t >= psi_p) {
                ++p;
                while (p < a.n && a.psi[p] == 0) ++p;
                p = uni_ll(p);
                if (p >= a.n) break;  // unreachable while g0 + B <= sum of Psi
                t = 0;
                psi_p = uni64(a.psi[p]);
                load_parent<T>(s, F + p * (long long)m, lane, par, am, om);
                for (int j = lane; j < m; j += 64) dg[j] = 0;
            } else {
                advance_digits(m, lane, om, dg);
            }
            wave_lds_sync();
        }
    }
    if (__any(ovf) && lane == 0) atomicOr((unsigned long long*)&a.ctr->overflow, 1ULL);
}

hipError_t launch_expand_sparse(int elem_bytes, const DevSystem& s, const ChunkArgs& a, hipStream_t st) {
    if (a.B <= 0) return hipSuccess;
    const int stride = ((kLdsBytesPerNeuron * s.m) + 15) & ~15;
    int wpb = 4;
    while (wpb > 1 && (size_t)wpb * stride > 64 * 1024) wpb >>= 1;
    if ((size_t)stride > 64 * 1024) return hipErrorInvalidValue;  // m too large for this form
    const int run = 16;
    const long long waves = (a.B + run - 1) / run;
    const unsigned blocks = (unsigned)((waves + wpb - 1) / wpb);
    const size_t lds = (size_t)wpb * stride;
    if (elem_bytes == 4)
        hipLaunchKernelGGL(k_expand_sparse<int32_t>, dim3(blocks), dim3(64 * wpb), lds, st, s, a, run, stride);
    else
        hipLaunchKernelGGL(k_expand_sparse<uint16_t>, dim3(blocks), dim3(64 * wpb), lds, st, s, a, run, stride);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Visited set.  Open addressing with linear probing over 64-bit entries
// (tag:32 | ref:32).  A child claims an empty slot with a CAS; a child that
// meets an entry with its tag compares the whole rows; an equal row of the
// current chunk with a larger index is replaced by atomicMin on the entry, so
// the entry ends at the first occurrence in canonical order.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_insert(int m, TableArgs a) {
    const int lane = threadIdx.x & 63;
    const long long b = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (b >= a.B) return;
    const u64 h = a.hash[b];
    const uint32_t tag = (uint32_t)(h >> 32);
    const uint32_t myref = kStageBase + (uint32_t)b;
    const u64 mine = ((u64)tag << 32) | myref;
    const T* row = (const T*)a.stage + b * (long long)m;
    u64 sl = h & a.slot_mask;
    for (u64 it = 0; it <= a.slot_mask; ++it) {
        u64 e = uni64(__hip_atomic_load(&a.table[sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (e == kEmpty) {
            u64 old = 0;
            if (lane == 0) old = atomicCAS(&a.table[sl], kEmpty, mine);
            old = uni64(__shfl(old, 0));
            if (old == kEmpty) {
                if (lane == 0) a.slot[b] = (uint32_t)sl;
                return;
            }
            e = old;
        }
        if (e != kTomb && (uint32_t)(e >> 32) == tag) {
            const uint32_t ref = (uint32_t)e;
            const T* other = ref < kStageBase ? (const T*)a.arena + (u64)ref * (u64)m
                                              : (const T*)a.stage + (u64)(ref - kStageBase) * (u64)m;
            bool diff = false;
            for (int j = lane; j < m; j += 64) diff |= (row[j] != other[j]);
            if (!__any(diff)) {
                if (lane == 0) {
                    if (ref >= kStageBase && myref < ref) atomicMin(&a.table[sl], mine);
                    a.slot[b] = (uint32_t)sl;
                }
                return;
            }
        }
        sl = (sl + 1) & a.slot_mask;
    }
    if (lane == 0) {
        a.slot[b] = 0;  // keep later kernels in bounds; the host reports the failure
        atomicOr((unsigned long long*)&a.ctr->probe_fail, 1ULL);
    }
}

hipError_t launch_insert(int elem_bytes, int m, const TableArgs& a, hipStream_t st) {
    if (a.B <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((a.B + 3) / 4);
    if (elem_bytes == 4) hipLaunchKernelGGL(k_insert<int32_t>, dim3(blocks), dim3(256), 0, st, m, a);
    else hipLaunchKernelGGL(k_insert<uint16_t>, dim3(blocks), dim3(256), 0, st, m, a);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_flags(const u64* __restrict__ table, const uint32_t* __restrict__ slot,
                                               long long B, uint32_t* __restrict__ flag) {
    const long long b = (long long)blockIdx.x * 256 + threadIdx.x;
    if (b >= B) return;
    flag[b] = ((uint32_t)table[slot[b]] == kStageBase + (uint32_t)b) ? 1u : 0u;
}

hipError_t launch_flags(const u64* table, const uint32_t* slot, long long B, uint32_t* flag, hipStream_t st) {
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_flags, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, table, slot, B, flag);
    return hipGetLastError();
}

// Commit the new children of a chunk in canonical order: rows below the
// level's limit are copied to the row store and their entries re-pointed at
// it; the rest (past a cap) become tombstones, i.e. are not recorded.
template <typename T>
__global__ __launch_bounds__(256) void k_commit(int m, CommitArgs a) {
    const int lane = threadIdx.x & 63;
    const long long b = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (b >= a.B) return;
    if (!a.flag[b]) return;
    const long long local = a.level_count + (long long)a.pos[b];
    const uint32_t sl = a.slot[b];
    const uint32_t tag = (uint32_t)(a.hash[b] >> 32);
    if (local < a.limit) {
        const long long A = a.level_base + local;
        const T* src = (const T*)a.stage + b * (long long)m;
        T* dst = (T*)a.arena + A * (long long)m;
        T* dst2 = a.row2 ? (T*)a.row2 + local * (long long)m : nullptr;
        for (int j = lane; j < m; j += 64) {
            const T v = src[j];
            dst[j] = v;
            if (dst2) dst2[j] = v;
        }
        if (lane == 0) {
            a.table[sl] = ((u64)tag << 32) | (uint32_t)A;
            a.row_slot[A] = sl;
            if (a.par_out) a.par_out[a.par_out_base + local] = (long long)a.cpar[b] + a.par_value_base;
            if (a.t_out) a.t_out[a.par_out_base + local] = (long long)a.ct[b];
            if (local == a.limit - 1) a.ctr->cap_g = (u64)b + 1;
        }
    } else if (lane == 0) {
        a.table[sl] = kTomb;
        atomicAdd(&a.ctr->tombs, 1ULL);
    }
}

hipError_t launch_commit(int elem_bytes, int m, const CommitArgs& a, hipStream_t st) {
    if (a.B <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((a.B + 3) / 4);
    if (elem_bytes == 4) hipLaunchKernelGGL(k_commit<int32_t>, dim3(blocks), dim3(256), 0, st, m, a);
    else hipLaunchKernelGGL(k_commit<uint16_t>, dim3(blocks), dim3(256), 0, st, m, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Maintenance kernels: table fill, unconditional insert of stored rows
// (C0 after a reset, or every row after a table rebuild), rollback of a
// level's rows, range check of rows handed in by the caller.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fill_u64(u64* __restrict__ p, long long n, u64 v) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_u64(u64* p, long long n, u64 v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void k_rows_insert(int m, u64* table, u64 slot_mask, const T* arena,
                                                     long long first, long long count, u64 hash_mask,
                                                     uint32_t* row_slot, DevCounters* ctr) {
    const int lane = threadIdx.x & 63;
    const long long q = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (q >= count) return;
    const long long A = first + q;
    const u64 h = row_hash_wave<T>(arena + A * (long long)m, m, lane) & hash_mask;
    const u64 mine = ((h >> 32) << 32) | (uint32_t)A;
    u64 sl = h & slot_mask;
    for (u64 it = 0; it <= slot_mask; ++it) {
        u64 old = 0;
        if (lane == 0) old = atomicCAS(&table[sl], kEmpty, mine);
        old = uni64(__shfl(old, 0));
        if (old == kEmpty) {
            if (lane == 0) row_slot[A] = (uint32_t)sl;
            return;
        }
        sl = (sl + 1) & slot_mask;
    }
    if (lane == 0) atomicOr((unsigned long long*)&ctr->probe_fail, 1ULL);
}

hipError_t launch_rows_insert(int elem_bytes, int m, u64* table, u64 slot_mask, const void* arena,
                              long long first, long long count, u64 hash_mask, uint32_t* row_slot,
                              DevCounters* ctr, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((count + 3) / 4);
    if (elem_bytes == 4)
        hipLaunchKernelGGL(k_rows_insert<int32_t>, dim3(blocks), dim3(256), 0, st, m, table, slot_mask,
                           (const int32_t*)arena, first, count, hash_mask, row_slot, ctr);
    else
        hipLaunchKernelGGL(k_rows_insert<uint16_t>, dim3(blocks), dim3(256), 0, st, m, table, slot_mask,
                           (const uint16_t*)arena, first, count, hash_mask, row_slot, ctr);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_rollback(const uint32_t* __restrict__ row_slot, u64* __restrict__ table,
                                                  long long first, long long count) {
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q < count) table[row_slot[first + q]] = kTomb;
}

hipError_t launch_rollback(const uint32_t* row_slot, u64* table, long long first, long long count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rollback, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, row_slot, table, first,
                       count);
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void k_check_rows(const T* __restrict__ rows, long long n, long long count_max,
                                                    DevCounters* ctr) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const long long v = (long long)rows[i];
    if (v < 0 || v > count_max) atomicOr((unsigned long long*)&ctr->overflow, 1ULL);
}

hipError_t launch_check_rows(int elem_bytes, const void* rows, long long n_elems, long long count_max,
                             DevCounters* ctr, hipStream_t st) {
    if (n_elems <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n_elems + 255) / 256);
    if (elem_bytes == 4)
        hipLaunchKernelGGL(k_check_rows<int32_t>, dim3(blocks), dim3(256), 0, st, (const int32_t*)rows, n_elems,
                           count_max, ctr);
    else
        hipLaunchKernelGGL(k_check_rows<uint16_t>, dim3(blocks), dim3(256), 0, st, (const uint16_t*)rows, n_elems,
                           count_max, ctr);
    return hipGetLastError();
}

}  // namespace snp
