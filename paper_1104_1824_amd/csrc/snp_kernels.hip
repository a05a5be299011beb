// gfx950 kernels of the breadth-first expansion of an SN P system's computation
// tree.  One level is: applicability and child counts Psi per parent, an
// exclusive prefix sum of Psi, then chunks of consecutive children g that are
// decoded (mixed radix), computed as C' = C + S.M (Equation next-config),
// hashed, deduplicated against the visited set and committed in order.
//
// Wave64 throughout: one wavefront per parent (Psi), per run of consecutive
// children (expand), or per child (insert / commit), lanes striding over the
// neurons of a row so that row loads and stores are contiguous.
#include "snp_device.hpp"

#include <algorithm>

namespace snp {

// ---------------------------------------------------------------------------
// Psi: per parent, number of valid spiking vectors (Algorithm 2 II-1/II-2):
// product over neurons of max(1, omega_n), saturated; 0 when no rule applies
// anywhere (halting) or when the parent exceeds the expansion count limit.
// ---------------------------------------------------------------------------
// b^e, saturated (square and multiply: at most 7 rounds for e < 128)
__device__ __forceinline__ u64 sat_pow(u64 b, uint32_t e) {
    u64 r = 1;
    while (e) {
        if (e & 1) r = sat_mul(r, b);
        e >>= 1;
        if (e) b = sat_mul(b, b);
    }
    return r;
}

// Saturating product over the wave (64-bit shuffles; only for radices above 4).
__device__ __forceinline__ u64 wave_satprod(u64 x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = sat_mul(x, __shfl_xor(x, o));
    return x;
}

// Psi of one parent (Algorithm 2: the product over neurons of the number of
// applicable rules, a neuron without one counting 1; 0 when no neuron has an
// applicable rule, or when a count exceeds expand_max), one wave, lane per
// neuron; halting = no rule applies anywhere.  The same pass counts the
// canonical children (the product of kappa, the canonical digits per neuron),
// the only ones the expansion computes.
struct PsiAcc {
    uint32_t c2 = 0, c3 = 0, c4 = 0;  // neurons with omega = 2, 3, 4
    uint32_t k2 = 0, k3 = 0, k4 = 0;  // neurons with kappa = 2, 3, 4
    bool any = false, over = false, big = false, kbig = false;
    u64 bigprod = 1, kbigprod = 1;
};

// Neuron j (< m) holding x spikes: its applicable rules, into the wave's
// tallies.  A parent is not expanded (Psi = 0, not halting) when a neuron
// holds more than expand_max spikes (the first mcount columns are spike
// counts), or when its output spike train (columns track, track + 1;
// track < 0: none) has two spikes: its number is generated.  With delays, a
// neuron that waits (wt >= 1: closed, or sending its delayed spikes) applies
// no rule, and the parent still has one child (the countdown moves on).
__device__ __forceinline__ void psi_add_neuron(PsiAcc& A, int x, int wt, int j, int m, int mcount, const int* nrp,
                                               const int4* rules, long long expand_max, int track) {
    int w = 0, k = 1;
    if (j < m) {
        if (wt <= 0) {
            const uint32_t am = neuron_applicable(x, nrp[j], nrp[j + 1], rules, w);
            k = kappa_of(am, w);
        }
        A.over |= (j < mcount && expand_max >= 0 && (long long)x > expand_max) || (j == track && x >= 2);
    }
    A.any |= (w > 0) || (wt > 0);
    A.c2 += __popcll(__ballot(w == 2));
    A.c3 += __popcll(__ballot(w == 3));
    A.c4 += __popcll(__ballot(w == 4));
    A.k2 += __popcll(__ballot(k == 2));
    A.k3 += __popcll(__ballot(k == 3));
    A.k4 += __popcll(__ballot(k == 4));
    if (w > 4) {
        A.big = true;
        A.bigprod = sat_mul(A.bigprod, (u64)w);
    }
    if (k > 4) {
        A.kbig = true;
        A.kbigprod = sat_mul(A.kbigprod, (u64)k);
    }
}

// Children of a parent: full (every valid spiking vector) and canonical.
struct PsiPair {
    u64 full, canon;
};

__device__ __forceinline__ PsiPair psi_finish(const PsiAcc& A, bool& halting) {
    const bool wany = __any(A.any);
    const bool wover = __any(A.over);
    u64 prod = sat_mul(sat_pow(2, A.c2 + 2 * A.c4), sat_pow(3, A.c3));  // 4^c4 = 2^(2 c4)
    if (__any(A.big)) prod = sat_mul(prod, wave_satprod(A.bigprod));
    u64 kprod = sat_mul(sat_pow(2, A.k2 + 2 * A.k4), sat_pow(3, A.k3));
    if (__any(A.kbig)) kprod = sat_mul(kprod, wave_satprod(A.kbigprod));
    halting = !wany;
    if (!wany || wover) return PsiPair{0, 0};
    return PsiPair{prod, kprod};
}

// Canonical children of the parent `row` whose child index t is below L
// (1 <= L <= 2^62).  Digits count from the most significant neuron; with
// (L - 1) written in the mixed radix of omega as digits l_n, a canonical child
// has t < L iff its digits are lexicographically <= those of L - 1, so the
// count is the sum, from the most significant neuron down to the first whose
// digit l_n is not canonical (included), of (canonical digits below l_n) x
// (product of kappa over the later neurons), plus one when every l_n is
// canonical.  Only the last 64 neurons with omega >= 2 can have a nonzero l_n
// (the 64 after any earlier one make its place value at least 2^64), so lane
// q takes the q-th of them from the end.  One wave, all lanes active.
template <typename T>
__device__ u64 canon_rank(const T* row, int m, const int* nrp, const int4* rules, const int* dlink, int mcount,
                          u64 L, int lane) {
    int cnt = 0;  // neurons taken so far (uniform)
    int myw = 1;
    uint32_t mycm = 1;
    for (int base = ((m - 1) >> 6) << 6; base >= 0 && cnt < 64; base -= 64) {
        const int j = base + lane;
        int w = 0;
        uint32_t am = 0;
        if (j < m && neuron_wait(row, dlink, mcount, j) <= 0)
            am = neuron_applicable((int)row[j], nrp[j], nrp[j + 1], rules, w);
        const u64 bm = __ballot(w >= 2);
        const int nb = __popcll(bm);
        // lane q (cnt <= q < cnt + nb) takes the (q - cnt)-th set bit of bm from the top
        const int pos = lane - cnt;
        const bool take = pos >= 0 && pos < nb;
        int src = 0;
        if (take) {
            u64 x = __builtin_bitreverse64(bm);  // bit i: lane 63 - i
            for (int k = 0; k < pos; ++k) x &= x - 1;
            src = 63 - __builtin_ctzll(x);
        }
        const int w_s = __shfl(w, src);
        const uint32_t am_s = (uint32_t)__shfl((int)am, src);
        if (take) {
            myw = w_s;
            mycm = am_s >> 16;
        }
        cnt = min(64, cnt + nb);
    }
    // place values over omega and kappa: products over the neurons after this one
    // (lanes below), exclusive, saturated
    const u64 wq = (u64)myw;
    u64 pw = wq, pk = (u64)__popc(mycm & ((1u << myw) - 1));
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const u64 yw = __shfl_up(pw, o), yk = __shfl_up(pk, o);
        if (lane >= o) {
            pw = sat_mul(pw, yw);
            pk = sat_mul(pk, yk);
        }
    }
    u64 placew = __shfl_up(pw, 1), placek = __shfl_up(pk, 1);
    if (lane == 0) placew = placek = 1;
    const u64 lim = L - 1;
    const int l = placew >= kPsiSat || placew > lim ? 0 : (int)((lim / placew) % wq);
    const uint32_t below = mycm & ((1u << l) - 1);
    const bool nc = !((mycm >> l) & 1u);
    const u64 ncm = __ballot(nc);
    const int qstop = ncm ? 63 - __clzll((long long)ncm) : -1;  // most significant non-canonical digit
    const u64 term = lane >= qstop ? sat_mul((u64)__popc(below), placek) : 0;
    return sat_add(wave_satsum(term), ncm ? 0 : 1);
}

template <typename T>
__device__ __forceinline__ PsiPair parent_psi(const T* row, int m, const int* nrp, const int4* rules,
                                              const int* dlink, int mcount, long long expand_max, int track,
                                              int lane, bool& halting) {
    PsiAcc A;
    for (int base = 0; base < m; base += 64) {
        const int j = base + lane;
        psi_add_neuron(A, j < m ? (int)row[j] : 0, j < m ? neuron_wait(row, dlink, mcount, j) : 0, j, m, mcount, nrp,
                       rules, expand_max, track);
    }
    PsiPair r = psi_finish(A, halting);
    // with 2^62 or more children some canonical ones may have t >= 2^62, past
    // what a level enumerates: count only those below
    if (r.full >= kPsiSat) r.canon = min(r.canon, canon_rank<T>(row, m, nrp, rules, dlink, mcount, kPsiSat, lane));
    return r;
}

// Rules and rule offsets staged in LDS when they fit (else read from global).
struct PsiTables {
    const int* nrp;
    const int4* rules;
};

template <bool TBL_LDS>
__device__ __forceinline__ PsiTables stage_psi_tables(const DevSystem& s, unsigned char* smem) {
    if constexpr (TBL_LDS) {
        int4* l_rules = (int4*)smem;
        int* l_nrp = (int*)(l_rules + s.r);
        for (int q = threadIdx.x; q < s.r; q += blockDim.x) l_rules[q] = s.rules[q];
        for (int q = threadIdx.x; q <= s.m; q += blockDim.x) l_nrp[q] = s.nrule_ptr[q];
        __syncthreads();
        return PsiTables{l_nrp, l_rules};
    } else {
        return PsiTables{s.nrule_ptr, s.rules};
    }
}

// Adds children counts (each <= 2^62) to ctr->psif_lo / psif_hi, split at bit
// 31 so that neither sum can wrap; the host joins and saturates them.
__device__ __forceinline__ void add_full_total(DevCounters* ctr, u64 lo, u64 hi) {
    if (lo) atomicAdd((unsigned long long*)&ctr->psif_lo, lo);
    if (hi) atomicAdd((unsigned long long*)&ctr->psif_hi, hi);
}

// S > 0: rows of at most 64 S entries, S strips of 64 held in registers, and
// the next parent's strips loaded while the current one is counted (its
// latency overlaps the work); S = 0: any width, one parent after another.
template <typename T, bool TBL_LDS, int S>
__global__ __launch_bounds__(256) void k_psi(DevSystem s, const T* __restrict__ F, long long n,
                                             long long expand_max, u64* __restrict__ psi, u64* __restrict__ psif,
                                             uint8_t* __restrict__ halt_flag, DevCounters* __restrict__ ctr,
                                             int parents_per_wave) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const PsiTables tb = stage_psi_tables<TBL_LDS>(s, smem);
    const long long w0 = ((long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * parents_per_wave;
    const long long pend = min(n, w0 + parents_per_wave);
    unsigned halting = 0;
    u64 flo = 0, fhi = 0;
    constexpr int SR = S > 0 ? S : 1;
    int dl[SR], x[SR], wt[SR];  // per strip: the wait column of the lane's neuron (-1: none), count, wait
    auto load = [&](long long p, int (&xx)[SR], int (&ww)[SR]) {
        const T* row = F + p * (long long)s.m;
#pragma unroll
        for (int q = 0; q < SR; ++q) {
            const int j = q * 64 + lane;
            xx[q] = j < s.m ? (int)row[j] : 0;
            ww[q] = dl[q] >= 0 ? (int)row[dl[q]] : 0;  // as neuron_wait
        }
    };
    if constexpr (S > 0) {
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int j = q * 64 + lane;
            dl[q] = (s.dlink && j < s.mcount) ? s.dlink[j] : -1;
        }
        if (w0 < pend) load(w0, x, wt);
    }
    for (long long p = w0; p < pend; ++p) {
        bool h;
        PsiPair v;
        if constexpr (S > 0) {
            int xn[SR], wn[SR];
#pragma unroll
            for (int q = 0; q < SR; ++q) xn[q] = wn[q] = 0;
            if (p + 1 < pend) load(p + 1, xn, wn);
            PsiAcc A;
#pragma unroll
            for (int q = 0; q < S; ++q)
                psi_add_neuron(A, x[q], wt[q], q * 64 + lane, s.m, s.mcount, tb.nrp, tb.rules, expand_max, s.track);
            v = psi_finish(A, h);
            if (v.full >= kPsiSat)
                v.canon = min(v.canon, canon_rank<T>(F + p * (long long)s.m, s.m, tb.nrp, tb.rules, s.dlink, s.mcount,
                                                     kPsiSat, lane));
#pragma unroll
            for (int q = 0; q < SR; ++q) {
                x[q] = xn[q];
                wt[q] = wn[q];
            }
        } else {
            v = parent_psi<T>(F + p * (long long)s.m, s.m, tb.nrp, tb.rules, s.dlink, s.mcount, expand_max, s.track,
                              lane, h);
        }
        const u64 full = min(v.full, s.psi_cap);
        if (lane == 0) {
            psi[p] = min(v.canon, s.psi_cap);
            psif[p] = full;
            halt_flag[p] = h ? 1 : 0;
        }
        halting += h ? 1u : 0u;
        flo += full & 0x7FFFFFFFull;
        fhi += full >> 31;
    }
    if (lane == 0 && halting) atomicAdd(&ctr->halting, (u64)halting);
    if (lane == 0) add_full_total(ctr, flo, fhi);
}

// Psi of at most kPsiScanSmall parents (m <= 64) and their exclusive prefix
// sums in one block: a wave per parent, then the block scans them from the
// base *base_dev (the children of the frontier before them,
// saturated), writing the new total to *total_dev and to ctr->psi_total.
constexpr int kPsiScanSmall = 16;  // one parent per wave: more would serialise their latency

template <typename T, bool TBL_LDS>
__global__ __launch_bounds__(1024) void k_psi_scan_small(DevSystem s, const T* __restrict__ F, int n,
                                                         long long expand_max, u64* __restrict__ psi,
                                                         u64* __restrict__ psif,
                                                         uint8_t* __restrict__ halt_flag, u64* __restrict__ off,
                                                         const u64* base_dev, u64* total_dev,
                                                         DevCounters* __restrict__ ctr) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ u64 wsum[16];
    __shared__ u64 l_psi[kPsiScanSmall];
    __shared__ u64 s_base;  // read before the total (possibly the same word) is written
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_base = base_dev ? *base_dev : 0;
    const PsiTables tb = stage_psi_tables<TBL_LDS>(s, smem);
    // m <= 64: a parent is one count per lane
    constexpr int kPre = (kPsiScanSmall + 15) / 16;
    unsigned halting = 0;
    const int m = s.m;
    for (int p0 = wid; p0 < n; p0 += 16 * kPre) {
        int xs[kPre];
#pragma unroll
        for (int q = 0; q < kPre; ++q) {
            const int p = p0 + 16 * q;
            xs[q] = (p < n && lane < m) ? (int)F[(long long)p * m + lane] : 0;
        }
#pragma unroll
        for (int q = 0; q < kPre; ++q) {
            const int p = p0 + 16 * q;
            if (p >= n) break;
            PsiAcc A;
            const int wt = lane < m ? neuron_wait(F + (long long)p * m, s.dlink, s.mcount, lane) : 0;
            psi_add_neuron(A, xs[q], wt, lane, m, s.mcount, tb.nrp, tb.rules, expand_max, s.track);
            bool h;
            PsiPair v2 = psi_finish(A, h);
            if (v2.full >= kPsiSat)
                v2.canon = min(v2.canon, canon_rank<T>(F + (long long)p * m, m, tb.nrp, tb.rules, s.dlink, s.mcount,
                                                       kPsiSat, lane));
            const u64 v = min(v2.canon, s.psi_cap);
            const u64 full = min(v2.full, s.psi_cap);
            if (lane == 0) {
                l_psi[p] = v;
                psi[p] = v;
                psif[p] = full;
                halt_flag[p] = h ? 1 : 0;
                add_full_total(ctr, full & 0x7FFFFFFFull, full >> 31);
            }
            halting += h ? 1u : 0u;
        }
    }
    if (lane == 0 && halting) atomicAdd(&ctr->halting, (u64)halting);
    __syncthreads();
    const int i = threadIdx.x;
    const u64 x = i < n ? l_psi[i] : 0;
    u64 incl = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const u64 y = __shfl_up(incl, o);
        if (lane >= o) incl = sat_add(incl, y);
    }
    u64 excl = __shfl_up(incl, 1);  // (not incl - x: sums may have saturated)
    if (lane == 0) excl = 0;
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    u64 pre = s_base;
    for (int w = 0; w < wid; ++w) pre = sat_add(pre, wsum[w]);
    if (i < n) off[i] = sat_add(pre, excl);
    if (i == 1023) {
        const u64 tot = sat_add(pre, incl);
        *total_dev = tot;
        ctr->psi_total = tot;
    }
}

hipError_t launch_psi(int elem_bytes, const DevSystem& s, const void* frontier, long long n,
                      long long expand_max, u64* psi, u64* psif, uint8_t* halt_flag, DevCounters* ctr,
                      hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const size_t tbl = (size_t)s.r * 16 + (size_t)(s.m + 1) * 4;
    const bool tbl_lds = tbl <= (size_t)(32 * 1024);
    // enough parents per wave to amortise the table staging, while filling the GPU
    int ppw = 1;
    while (ppw < 16 && (long long)ppw * 2 * 4 * 2048 <= n) ppw <<= 1;
    const long long waves = (n + ppw - 1) / ppw;
    const unsigned blocks = (unsigned)((waves + 3) / 4);
    const size_t lds = tbl_lds ? tbl : 0;
    const int strips = s.m <= 64 ? 1 : s.m <= 128 ? 2 : s.m <= 256 ? 4 : 0;
#define SNP_PSI_S(TT, L, SS)                                                                                       \
    hipLaunchKernelGGL((k_psi<TT, L, SS>), dim3(blocks), dim3(256), lds, st, s, (const TT*)frontier, n, expand_max, \
                       psi, psif, halt_flag, ctr, ppw)
#define SNP_PSI(TT, L)                              \
    do {                                            \
        if (strips == 1) SNP_PSI_S(TT, L, 1);       \
        else if (strips == 2) SNP_PSI_S(TT, L, 2);  \
        else if (strips == 4) SNP_PSI_S(TT, L, 4);  \
        else SNP_PSI_S(TT, L, 0);                   \
    } while (0)
    if (elem_bytes == 4) {
        if (tbl_lds) SNP_PSI(int32_t, true);
        else SNP_PSI(int32_t, false);
    } else {
        if (tbl_lds) SNP_PSI(uint16_t, true);
        else SNP_PSI(uint16_t, false);
    }
#undef SNP_PSI
#undef SNP_PSI_S
    return hipGetLastError();
}

bool psi_scan_fits(const DevSystem& s, long long n) { return s.m <= 64 && n > 0 && n <= kPsiScanSmall; }

hipError_t launch_psi_scan_small(int elem_bytes, const DevSystem& s, const void* frontier, long long n,
                                 long long expand_max, u64* psi, u64* psif, uint8_t* halt_flag, u64* off,
                                 const u64* base_dev, u64* total_dev, DevCounters* ctr, hipStream_t st) {
    if (!psi_scan_fits(s, n)) return hipErrorInvalidValue;
    const size_t tbl = (size_t)s.r * 16 + (size_t)(s.m + 1) * 4;
    const bool tbl_lds = tbl <= (size_t)(32 * 1024);
    const size_t lds = tbl_lds ? tbl : 0;
#define SNP_PSS(TT, L)                                                                                     \
    hipLaunchKernelGGL((k_psi_scan_small<TT, L>), dim3(1), dim3(1024), lds, st, s, (const TT*)frontier, (int)n, \
                       expand_max, psi, psif, halt_flag, off, base_dev, total_dev, ctr)
    if (elem_bytes == 4) {
        if (tbl_lds) SNP_PSS(int32_t, true);
        else SNP_PSS(int32_t, false);
    } else {
        if (tbl_lds) SNP_PSS(uint16_t, true);
        else SNP_PSS(uint16_t, false);
    }
#undef SNP_PSS
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
                                                    long long ntiles, u64* total, const u64* base_dev,
                                                    u64* total_copy) {
    __shared__ V wsum[16];
    __shared__ V carry_s;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry_s = base_dev ? (V)*base_dev : (V)0;
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
    if (threadIdx.x == 0) {
        *total = (u64)carry_s;
        if (total_copy) *total_copy = (u64)carry_s;
    }
}

template <typename V, bool SAT>
__global__ __launch_bounds__(256) void k_scan_add(V* __restrict__ out, const V* __restrict__ pre, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = vadd<V, SAT>(pre[i / kScanTile], out[i]);
}

long long scan_tiles(long long n) { return (n + kScanTile - 1) / kScanTile; }

// out[i] = base + sum of in[0 .. i); *total = base + sum of in, where base is
// read on the device (*base_dev, 0 when null) and may be the same word as total.
// Up to this many elements one block scans them directly (one pass of
// k_scan_sums with the carried base): one launch instead of two or three.
constexpr long long kSmallScan = 1024;

template <typename V, bool SAT>
static hipError_t scan_impl(const V* in, V* out, long long n, V* tile_sums, V* tile_pre, u64* total,
                            const u64* base_dev, u64* total_copy, hipStream_t st) {
    if (n <= kSmallScan) {
        hipLaunchKernelGGL((k_scan_sums<V, SAT>), dim3(1), dim3(1024), 0, st, in, out, n, total, base_dev,
                           total_copy);
        return hipGetLastError();
    }
    const long long nt = scan_tiles(n);
    if (nt > 0) hipLaunchKernelGGL((k_scan_tiles<V, SAT>), dim3((unsigned)nt), dim3(256), 0, st, in, out, tile_sums, n);
    hipLaunchKernelGGL((k_scan_sums<V, SAT>), dim3(1), dim3(1024), 0, st, tile_sums, tile_pre, nt, total, base_dev,
                       total_copy);
    if (nt > 1 || (nt == 1 && base_dev))
        hipLaunchKernelGGL((k_scan_add<V, SAT>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, out, tile_pre, n);
    return hipGetLastError();
}

hipError_t launch_scan_u64(const u64* in, u64* out, long long n, u64* tile_sums, u64* tile_pre, u64* total,
                           const u64* base_dev, u64* total_copy, hipStream_t st) {
    return scan_impl<u64, true>(in, out, n, tile_sums, tile_pre, total, base_dev, total_copy, st);
}



__global__ __launch_bounds__(256) void k_count_flags(const uint8_t* __restrict__ f, long long n, u64* out) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    const bool v = i < n && f[i] != 0;
    const u64 bm = __ballot(v);
    if ((threadIdx.x & 63) == 0 && bm) atomicAdd(out, (u64)__popcll(bm));
}

hipError_t launch_count_flags(const uint8_t* flags, long long n, u64* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_flags, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, flags, n, out);
    return hipGetLastError();
}

// The same count over flags [0, cap_par + 1), and the sum of all children
// of parents [0, cap_par), when the pass's commit filled the cap (cap_g != 0),
// else nothing; n bounds the flags computed so far.
__global__ __launch_bounds__(256) void k_count_flags_cap(const uint8_t* __restrict__ f, const u64* __restrict__ psif,
                                                         long long n, DevCounters* ctr) {
    if (ctr->cap_g == 0) return;
    const long long cp = (long long)ctr->cap_par;
    const long long lim = min(n, cp + 1);
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    const bool v = i < lim && f[i] != 0;
    const u64 full = i < min(n, cp) ? psif[i] : 0;
    const u64 bm = __ballot(v);
    const u64 flo = wave_sum_u64(full & 0x7FFFFFFFull), fhi = wave_sum_u64(full >> 31);
    if ((threadIdx.x & 63) == 0) {
        if (bm) atomicAdd((unsigned long long*)&ctr->count, (u64)__popcll(bm));
        if (flo) atomicAdd((unsigned long long*)&ctr->capf_lo, flo);
        if (fhi) atomicAdd((unsigned long long*)&ctr->capf_hi, fhi);
    }
}

hipError_t launch_count_flags_cap(const uint8_t* flags, const u64* psif, long long n, DevCounters* ctr,
                                  hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_flags_cap, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, flags, psif, n, ctr);
    return hipGetLastError();
}

// Child budget (one block).  The parents' full child counts are summed in
// order to find the parent p_b holding child g = budget - 1; the canonical
// children before the budget are then off[p_b] plus the canonical children of
// p_b with child index below budget - (all children of the parents before
// p_b), from canon_rank.  With no more than `budget` children in the prefix
// the end stays the prefix's canonical total.
template <typename T>
__global__ __launch_bounds__(1024) void k_budget_clip(DevSystem s, const T* __restrict__ F, long long n,
                                                      const u64* __restrict__ psif, const u64* __restrict__ off,
                                                      const u64* __restrict__ total, u64 budget, u64* tend,
                                                      DevCounters* ctr) {
    __shared__ u64 wsum[16];
    __shared__ u64 s_carry;
    __shared__ long long s_pb;
    __shared__ u64 s_before;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (threadIdx.x == 0) {
        s_carry = 0;
        s_pb = -1;
    }
    __syncthreads();
    for (long long b = 0; b < n; b += 1024) {
        const long long i = b + threadIdx.x;
        const u64 x = i < n ? psif[i] : 0;
        u64 incl = x;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const u64 y = __shfl_up(incl, o);
            if (lane >= o) incl = sat_add(incl, y);
        }
        u64 excl = __shfl_up(incl, 1);
        if (lane == 0) excl = 0;
        if (lane == 63) wsum[wid] = incl;
        __syncthreads();
        u64 pre = s_carry;
        for (int w = 0; w < wid; ++w) pre = sat_add(pre, wsum[w]);
        const u64 before = sat_add(pre, excl);  // children of the parents before i
        // parent i holds child budget - 1 when before < budget <= before + x
        if (i < n && x > 0 && before < budget && budget <= sat_add(before, x)) {
            s_pb = i;
            s_before = before;
        }
        __syncthreads();
        if (threadIdx.x == 1023) s_carry = sat_add(pre, incl);
        __syncthreads();
        if (s_pb >= 0) break;
    }
    const u64 T0 = *total;
    if (s_pb < 0) {  // the prefix holds no more than budget children
        if (threadIdx.x == 0) {
            *tend = T0;
            ctr->tend = T0;
        }
        return;
    }
    if (wid == 0) {
        const long long pb = s_pb;
        const u64 rank = canon_rank<T>(F + pb * (long long)s.m, s.m, s.nrule_ptr, s.rules, s.dlink, s.mcount,
                                       budget - s_before, lane);
        if (lane == 0) {
            const u64 e = min(T0, sat_add(off[pb], rank));
            *tend = e;
            ctr->tend = e;
            ctr->bud_par = (u64)pb + 1;
        }
    }
}

hipError_t launch_budget_clip(int elem_bytes, const DevSystem& s, const void* frontier, long long n,
                              const u64* psif, const u64* off, const u64* total, u64 budget, u64* tend,
                              DevCounters* ctr, hipStream_t st) {
    if (elem_bytes == 4)
        hipLaunchKernelGGL(k_budget_clip<int32_t>, dim3(1), dim3(1024), 0, st, s, (const int32_t*)frontier, n, psif,
                           off, total, budget, tend, ctr);
    else
        hipLaunchKernelGGL(k_budget_clip<uint16_t>, dim3(1), dim3(1024), 0, st, s, (const uint16_t*)frontier, n,
                           psif, off, total, budget, tend, ctr);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Expansion, sparse form.  Every wave owns a run of consecutive canonical
// children g0 + b0 .. g0 + b0 + run - 1.  Per wave, LDS holds the parent row,
// the applicable-rule mask (with the canonical digits) and count omega of
// every neuron, the current canonical digit of every neuron, and the
// consumption c and production p of every neuron's fired rule.  When the rule
// table and the in-synapse lists are small they are staged once per block in
// LDS as well, so the per-child loop touches no global memory except the row
// it writes.
//
//   decode (once per run): place value of each lane's block of neurons is a
//     suffix product of kappa across lanes; canonical digits follow by division.
//   advance (per child): add one to the mixed-radix number of canonical
//     digits: the last neuron with kappa >= 2 whose digit is below kappa - 1
//     steps up and every later neuron with kappa >= 2 resets to 0; only those
//     neurons refresh their fired (c, p).  Past the last canonical child of a
//     parent the wave moves to the next parent with one, digits all 0.
//   child (per child): C'[d] = C[d] - c(fired rule of d) + sum over in-synapses
//     (s, d) of p(fired rule of s): the nonzero entries of column d of S.M;
//     its child index t from the digits (child_index).
// ---------------------------------------------------------------------------
constexpr int kLdsBytesPerNeuron = 4 /*par*/ + 4 /*c:p*/ + 4 /*mask*/ + 1 /*omega*/ + 1 /*digit*/;
constexpr int kTableLdsLimit = 24 * 1024;

struct Tables {
    const int* nrp;    // [m+1]
    const int4* rules; // [r]
    const int* inp;    // [m+1]
    const int* ins;    // [nnz]
    const u64* R;      // [m] hash weights
};

// Fired rule of neuron j (canonical digit eg[j]) packed as (c << 16) | q, q
// the spikes it sends at this step (c, q <= 65535, checked at load); 0 when it
// fires nothing.  Without delays q = p of the fired rule.  With delays (dx
// non-null): q = p for a rule without delay, the pending spikes of a neuron
// whose wait ends now, else 0; and dx[j] = (closed << 31) | (d << 16) | p of
// the fired rule (0 when none), closed meaning that spikes sent to j at this
// step are lost (it fires a rule with a delay, or waits two steps or more).
__device__ __forceinline__ void set_fired(const Tables& tb, const DevSystem& s, int j, const uint8_t* om,
                                          const uint32_t* am, const uint8_t* eg, const int* par, uint32_t* cp,
                                          uint32_t* dx) {
    uint32_t c = 0, w = 0;
    if (om[j]) {
        const int d = canon_digit(am[j], om[j], eg[j]);
        const int4 R = tb.rules[tb.nrp[j] + nth_bit(am[j] & 0xFFFFu, d)];
        c = (uint32_t)R.z;
        w = (uint32_t)R.w;
    }
    if (!dx) {
        cp[j] = (c << 16) | w;
        return;
    }
    int wait = 0, pend = 0;
    if (j < s.mcount) {
        const int col = s.dlink[j];
        if (col >= 0) {
            wait = par[col];
            pend = par[col + 1];
        }
    }
    const uint32_t d = w >> 16, p = w & 0xFFFFu;
    const uint32_t q = (om[j] && d == 0) ? p : (wait == 1 ? (uint32_t)pend : 0u);
    const bool closed = d >= 1 || wait >= 2;
    cp[j] = (c << 16) | q;
    dx[j] = (closed ? 0x80000000u : 0u) | w;
}

// A parent's row into LDS with every neuron's applicable rules and omega (a
// neuron that waits, with delays, has none).
template <typename T>
__device__ __forceinline__ void load_parent(const Tables& tb, const DevSystem& s, int m, const T* row, int lane,
                                            int* par, uint32_t* am, uint8_t* om) {
    for (int j = lane; j < m; j += 64) {
        const int x = (int)row[j];
        par[j] = x;
        int w = 0;
        am[j] = neuron_wait(row, s.dlink, s.mcount, j) > 0 ? 0u
                                                           : neuron_applicable(x, tb.nrp[j], tb.nrp[j + 1], tb.rules, w);
        om[j] = (uint8_t)w;
    }
}

// State column j (>= dfirst) of a child, with delays: a neuron firing a rule
// with delay d >= 1 waits d steps to send its p spikes; otherwise the wait
// counts down, and the pending spikes stay until the step that sends them.
__device__ __forceinline__ long long delay_state(const DevSystem& s, const int* par, const uint32_t* dx, int j) {
    const int n = s.dlink[j];
    const int col = s.dlink[n];
    const uint32_t f = dx[n] & 0x7FFFFFFFu;
    const long long wait = par[col], pend = par[col + 1];
    if (j == col) return (f >> 16) ? (long long)(f >> 16) : (wait >= 1 ? wait - 1 : 0);
    return (f >> 16) ? (long long)(f & 0xFFFFu) : (wait >= 2 ? pend : 0);
}

// The output neuron's spike train of a child (column j = track: spikes sent
// to the environment, at most 2 counted; j = track + 1: steps from the first
// to the second), from the parent's (par) and the q spikes the output neuron
// sends out at this step (cp: (c << 16) | q).
__device__ __forceinline__ long long spike_train(const DevSystem& s, const int* par, const uint32_t* cp, int j) {
    const long long q = (long long)(cp[s.out] & 0xFFFFu);
    const long long env = par[s.track], el = par[s.track + 1];
    if (j == s.track) return env == 0 ? min(2LL, q) : env == 1 ? min(2LL, 1 + q) : env;
    return env == 0 ? 0 : env == 1 ? el + 1 : el;
}

__host__ __device__ __forceinline__ size_t table_lds_bytes(const DevSystem& s, int nnz) {
    return ((size_t)((s.m + 1) & ~1) * 8 + (size_t)s.r * 16 + (size_t)(s.m + 1) * 8 + (size_t)nnz * 4 + 15) &
           ~(size_t)15;
}

// Bytes of a wave's LDS in the sparse form: par, cp, am (4 B each), omega and
// digit (1 B each) per column, and with delays dx (4 B, 4-aligned) per column.
__host__ __device__ __forceinline__ int sparse_dx_offset(int m) { return (kLdsBytesPerNeuron * m + 3) & ~3; }
__host__ __device__ __forceinline__ int sparse_wave_stride(int m, bool delay) {
    return ((delay ? sparse_dx_offset(m) + 4 * m : kLdsBytesPerNeuron * m) + 15) & ~15;
}

template <typename T, bool TBL_LDS, bool DELAY>
__global__ __launch_bounds__(256) void k_expand_sparse(DevSystem s, ChunkArgs a, int run, int wave_stride) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const int m = s.m;
    Tables tb{s.nrule_ptr, s.rules, s.in_ptr, s.in_src, s.R};
    unsigned char* wave_base = smem;
    if constexpr (TBL_LDS) {
        // hash weights, rule table and in-synapse lists, shared by the block's waves
        u64* l_R = (u64*)smem;
        int4* l_rules = (int4*)(l_R + ((m + 1) & ~1));
        int* l_nrp = (int*)(l_rules + s.r);
        int* l_inp = l_nrp + (m + 1);
        int* l_ins = l_inp + (m + 1);
        const int nnz = s.in_ptr[m];
        for (int q = threadIdx.x; q < m; q += blockDim.x) l_R[q] = s.R[q];
        for (int q = threadIdx.x; q < s.r; q += blockDim.x) l_rules[q] = s.rules[q];
        for (int q = threadIdx.x; q <= m; q += blockDim.x) {
            l_nrp[q] = s.nrule_ptr[q];
            l_inp[q] = s.in_ptr[q];
        }
        for (int q = threadIdx.x; q < nnz; q += blockDim.x) l_ins[q] = s.in_src[q];
        __syncthreads();
        tb = Tables{l_nrp, l_rules, l_inp, l_ins, l_R};
        wave_base = smem + table_lds_bytes(s, nnz);
    }
    const long long wave = (long long)blockIdx.x * (blockDim.x >> 6) + wid;
    const long long b0 = wave * run;
    const u64 tot = *a.Tdev;
    const long long Beff = tot > a.g0 ? (long long)min((u64)a.B, tot - a.g0) : 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctr->beff = (u64)Beff;
    if (b0 >= Beff) return;
    unsigned char* base = wave_base + (size_t)wid * wave_stride;
    int* par = (int*)base;
    uint32_t* cp = (uint32_t*)(par + m);
    uint32_t* am = cp + m;
    uint8_t* om = (uint8_t*)(am + m);
    uint8_t* eg = om + m;
    uint32_t* dx = DELAY ? (uint32_t*)(base + sparse_dx_offset(m)) : nullptr;
    const T* F = (const T*)a.frontier;
    T* stage = (T*)a.stage;
    const int cnt = (int)min((long long)run, Beff - b0);

    // parent of the first child: last p with off[p] <= g (it has a canonical
    // child), found by a 64-ary search: every lane probes one point per round
    const u64 g = a.g0 + (u64)b0;
    long long lo = 0, hi = a.n;  // off[lo] <= g; the answer lies in [lo, hi)
    while (hi - lo > 1) {
        const long long step = (hi - lo + 63) / 64;
        const long long idx = lo + (long long)lane * step;
        const bool ok = idx < hi && a.off[idx] <= g;
        const u64 mask = __ballot(ok);
        const int last = 63 - __clzll((long long)mask);
        lo = lo + (long long)last * step;
        hi = min(hi, lo + step);
    }
    long long p = uni_ll(lo);
    u64 u = uni64(g - a.off[p]);
    u64 psi_p = uni64(a.psi[p]);
    load_parent<T>(tb, s, m, F + p * (long long)m, lane, par, am, om);
    wave_lds_sync();
    u64 place_w = digit_place(m, lane, om);  // place values of child indices (omega)
    canon_decode(m, lane, u, om, am, eg, canon_place(m, lane, om, am));
    wave_lds_sync();
    for (int j = lane; j < m; j += 64) set_fired(tb, s, j, om, am, eg, par, cp, dx);

    bool ovf = false;
    for (int k = 0; k < cnt; ++k) {
        const long long b = b0 + k;
        wave_lds_sync();
        u64 h = 0;
        T* out = stage + b * (long long)m;
        for (int j = lane; j < m; j += 64) {
            long long v = (long long)par[j] - (long long)(cp[j] >> 16);
            if (!DELAY || !(dx[j] >> 31)) {  // with delays, spikes sent to a closed neuron are lost
                const int e1 = tb.inp[j + 1];
                for (int e = tb.inp[j]; e < e1; ++e) v += cp[tb.ins[e]] & 0xFFFFu;
            }
            if (DELAY && j >= s.dfirst) v = delay_state(s, par, dx, j);
            else if (s.track >= 0 && j >= s.track) v = spike_train(s, par, cp, j);
            ovf |= (v < 0) | (v > s.count_max);
            out[j] = (T)v;
            h += hterm((uint32_t)v, tb.R[j]);
        }
        h = wave_sum_u64(h);
        const u64 t = child_index(m, lane, om, am, eg, place_w);
        if (lane == 0) {
            a.hash[b] = fmix64(h) & a.hash_mask;
            a.cpar[b] = (int)p;
            a.ct[b] = t;
        }
        if (k + 1 < cnt) {
            ++u;
            wave_lds_sync();  // every lane has read cp and eg before they change
            if (u >= psi_p) {
                ++p;
                while (p < a.n && a.psi[p] == 0) ++p;
                p = uni_ll(p);
                if (p >= a.n) break;  // unreachable while g0 + B <= sum of Psi
                u = 0;
                psi_p = uni64(a.psi[p]);
                load_parent<T>(tb, s, m, F + p * (long long)m, lane, par, am, om);
                wave_lds_sync();
                place_w = digit_place(m, lane, om);
                for (int j = lane; j < m; j += 64) {
                    eg[j] = 0;
                    set_fired(tb, s, j, om, am, eg, par, cp, dx);
                }
            } else {
                int myJ = -1;
                for (int j = lane; j < m; j += 64) {
                    const int kp = kappa_of(am[j], om[j]);
                    if (kp >= 2 && eg[j] < kp - 1) myJ = j;
                }
                const int J = wave_max_i32(myJ);
                for (int j = lane; j < m; j += 64) {
                    const int kp = kappa_of(am[j], om[j]);
                    if (j == J) {
                        eg[j] = (uint8_t)(eg[j] + 1);
                        set_fired(tb, s, j, om, am, eg, par, cp, dx);
                    } else if (kp >= 2 && j > J) {
                        eg[j] = 0;
                        set_fired(tb, s, j, om, am, eg, par, cp, dx);
                    }
                }
            }
        }
    }
    if (__any(ovf) && lane == 0) atomicOr((unsigned long long*)&a.ctr->overflow, 1ULL);
}

// ---------------------------------------------------------------------------
// Expansion, one neuron per lane (m <= 64, in-degree <= kLaneMaxIn).  A wave
// walks runs of consecutive canonical children; a run is cut into segments of
// one parent each.  Within a segment u_a .. u_b only the canonical digits of
// V, the neurons with kappa >= 2 from the most significant digit where u_a
// and u_b differ on, ever change, so:
//   * the first child (the reference) is computed in full, by a pull over the
//     in-synapses (ds_bpermute) with lane j holding neuron j;
//   * every odometer step over V has one table row U (lane j: the change to
//     neuron j) in LDS, with its hash change and its child-index change (both
//     are linear in the digits) kept in the row's lane;
//   * for up to 64 children at a time, lane l finds the step from child l to
//     l + 1 from the digits of its V value, prefix sums over the lanes give
//     every child's hash and child index, and the hash, parent and child index
//     of the 64 children are stored at once;
//   * then the children's rows follow one after the other: one LDS row added
//     and one coalesced row store each.
// Counts are kept offset by 2^16 in 32 bits, so negative and too large values
// stay ordered for the range check (a running minimum and maximum).  A
// segment whose tables would not fit is cut in half until they do (a single
// child needs none).  The next parent's row and the Psi of the next 64
// parents are fetched ahead of use.
// ---------------------------------------------------------------------------
constexpr int kLaneMaxIn = 16;
constexpr int kLaneTab = 32;              // table rows per wave: sum of kappa over V
constexpr uint32_t kLaneOff = 1u << 16;   // count offset (c <= 65535)

// Ends the wait for a loaded register here, so that the per-child loop never
// waits on the row stores it has in flight (one counter covers both).
__device__ __forceinline__ void settle(int v) { asm volatile("" ::"v"(v)); }

// y / w for y < 2^20 and 2 <= w <= 16: a float reciprocal estimate is within
// one of the quotient there, and one correction makes it exact.
__device__ __forceinline__ uint32_t udiv_small(uint32_t y, uint32_t w) {
    uint32_t q = (uint32_t)((float)y * __builtin_amdgcn_rcpf((float)w));
    const int r = (int)(y - q * w);
    return r < 0 ? q - 1 : (r >= (int)w ? q + 1 : q);
}

// c, p and H(M_k) of the rule canonical digit e picks (0 when no rule applies).
__device__ __forceinline__ void lane_fired(const int4* rules, const u64* hrow, int r0, uint32_t am, int om, int e,
                                           uint32_t& c, uint32_t& p, u64& hv) {
    c = 0;
    p = 0;
    hv = 0;
    if (om > 0) {
        const int k = r0 + nth_bit(am & 0xFFFFu, canon_digit(am, om, e));
        const int4 R = rules[k];
        c = (uint32_t)R.z;
        p = (uint32_t)R.w;
        hv = hrow[k];
    }
}

__device__ __forceinline__ u64 readlane64(u64 v, int j) {
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, j);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), j);
    return ((u64)hi << 32) | lo;
}

// Product over the lanes after this one of factors >= 1, saturated at 2^62
// (lane 63: 1).
__device__ __forceinline__ u64 wave_after_prod64(u64 w) {
    u64 incl = w;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const u64 y = __shfl_down(incl, o);
        if (__lane_id() + o < 64) incl = sat_mul(incl, y);
    }
    const u64 a64 = __shfl_down(incl, 1);
    return __lane_id() == 63 ? 1 : a64;
}

template <typename T>
__global__ __launch_bounds__(256) void k_expand_lane(DevSystem s, ChunkArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    int4* l_rules = (int4*)smem;
    u64* l_hM = (u64*)(l_rules + s.r);
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    uint32_t* l_tab = (uint32_t*)(smem + (size_t)s.r * 24) + (size_t)wid * (kLaneTab * 64);
    const int m = s.m;
    const bool act = lane < m;
    const int kin = s.max_in;
    // Per-lane constants, loaded unconditionally (clamped index, then a
    // select) so that no load waits inside a branch.
    const int jl = min(lane, m - 1);
    int r0 = s.nrule_ptr[jl], r1 = s.nrule_ptr[jl + 1];
    u64 Rj = s.R[jl];
    // in-synapse sources of neuron `lane` from the lane-major table (-1: none),
    // independent of the other loads
    int saddr[kLaneMaxIn];
#pragma unroll
    for (int e = 0; e < kLaneMaxIn; ++e) saddr[e] = e < kin ? s.in_lane[e * 64 + lane] : -1;
    if (!act) r0 = r1 = 0, Rj = 0;
    // The chunk ends at the children known on the device; the grid strides
    // over runs of consecutive children, about one run per wave.
    const u64 tot = *a.Tdev;
    const long long Beff = tot > a.g0 ? (long long)min((u64)a.B, tot - a.g0) : 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctr->beff = (u64)Beff;
    const long long wpb = blockDim.x >> 6;
    const long long nwaves = (long long)gridDim.x * wpb;
    const int run = (int)max(4LL, min(4096LL, (Beff + nwaves - 1) / nwaves));
    const long long nruns = (Beff + run - 1) / run;
    if ((long long)blockIdx.x * wpb >= nruns) return;  // the whole block
    for (int q = threadIdx.x; q < s.r; q += blockDim.x) {
        l_rules[q] = s.rules[q];
        l_hM[q] = s.hM[q];
    }
    __syncthreads();
    const long long wave0 = (long long)blockIdx.x * wpb + wid;
    if (wave0 >= nruns) return;

    // in-synapses: ds_bpermute byte addresses, which of them exist, and a
    // mask of the source neurons
    u64 inmask = 0;
    uint32_t emask = 0;
#pragma unroll
    for (int e = 0; e < kLaneMaxIn; ++e) {
        const bool ok = saddr[e] >= 0;
        if (ok) inmask |= 1ULL << saddr[e];
        emask |= ok ? 1u << e : 0u;
        saddr[e] = ok ? 4 * saddr[e] : 0;
    }

    const T* F = (const T*)a.frontier;
    T* stage = (T*)a.stage;
    const long long n = a.n;
    const uint32_t hi_ok = (uint32_t)s.count_max + kLaneOff;
    uint32_t vmin = kLaneOff, vmax = kLaneOff;  // range of the stored counts (offset)
    for (long long rw = wave0; rw < nruns; rw += nwaves) {
        const long long b0 = rw * run;
        const int cnt = (int)min((long long)run, Beff - b0);
        // parent of the first child (64-ary search, one probe per lane per round)
        const u64 g = a.g0 + (u64)b0;
        long long lo = 0, hi = n;
        while (hi - lo > 1) {
            const long long step = (hi - lo + 63) / 64;
            const long long idx = lo + (long long)lane * step;
            const bool ok = idx < hi && a.off[idx] <= g;
            const u64 mask = __ballot(ok);
            lo = lo + (long long)(63 - __clzll((long long)mask)) * step;
            hi = min(hi, lo + step);
        }

        // Psi window: parents pbase .. pbase + 63; the current parent is lane cur
        long long p = uni_ll(lo);
        long long pbase = p;
        int cur = 0;
        u64 pw = a.psi[min(pbase + lane, n - 1)];
        if (pbase + lane >= n) pw = 0;
        u64 u = uni64(g - a.off[p]);
        int x = (int)F[p * (long long)m + jl];
        settle(x);
        u64 psi_p = uni64(__shfl(pw, 0));
        // next parent with children, and its row fetched ahead
        long long pf_p = -1;
        int pf_x = 0;
        {
            const u64 nb = __ballot(pw > 0 && lane > cur);
            if (nb) {
                pf_p = pbase + __builtin_ctzll(nb);
                pf_x = (int)F[pf_p * (long long)m + jl];
            }
        }
        uint32_t am;
        int om;
        am = neuron_applicable(x, r0, r1, l_rules, om);
        // kappa of this lane's neuron and the place value of its digit in the
        // child index (product of max(1, omega) over later lanes)
        int kp = kappa_of(am, om);
        u64 place_w = wave_after_prod64((u64)max(1, om));

        int k = 0;
        while (k < cnt) {
            // ---- a segment: canonical children u .. u + len - 1 of parent p ----
            int len = (int)min((u64)(cnt - k), psi_p - u);
            // place value of lane j over canonical digits: product of kappa over
            // later lanes.  Digit j of canonical index y is (y / place_j) mod
            // kappa_j.  When the parent's canonical count fits 32 bits so does
            // every index of the segment, and place values saturated at 2^32 - 1
            // still compare right with them: the whole decomposition then runs
            // in 32-bit arithmetic.
            const bool narrow = psi_p <= 0xFFFFFFFFull;  // uniform
            const uint32_t w1 = (uint32_t)kp;
            u64 after = 1;
            if (narrow) after = wave_after_prod_sat32(w1);
            else after = wave_after_prod64(w1);
            auto quot = [&](u64 y) -> u64 {
                if (narrow) {
                    const uint32_t y32 = (uint32_t)y, a32 = (uint32_t)after;
                    return a32 > y32 ? 0u : y32 / a32;
                }
                return after > y ? 0 : y / after;
            };
            const u64 qa = quot(u);
            const int dg0 = narrow ? (int)((uint32_t)qa % w1) : (int)(qa % w1);
            // V: neurons with kappa >= 2 from the most significant digit that
            // changes inside the segment; halve the segment until its tables fit
            u64 vmask;
            int nt;
            for (;;) {
                const u64 ub = u + (u64)(len - 1);
                const u64 qb = quot(ub);
                const u64 dif = __ballot(act && qa != qb);
                const int jstar = dif ? __builtin_ctzll(dif) : 64;
                vmask = __ballot(act && kp >= 2 && lane >= jstar);
                nt = (int)wave_sum_u32((vmask >> lane) & 1 ? (uint32_t)kp : 0u);
                if (nt <= kLaneTab && __popcll(vmask) <= 16) break;
                len = (len + 1) / 2;
            }
            const bool inV = (vmask >> lane) & 1;
            // table base of every V lane: kappa summed over earlier V lanes
            const uint32_t tb_incl = wave_incl_u32(inV ? (uint32_t)kp : 0u);
            const int tbase = (int)tb_incl - (inV ? kp : 0);
            // the reference child (canonical digits dg0) in full, with its child index
            int dg = dg0;
            uint32_t c, pp;
            u64 hv;
            lane_fired(l_rules, l_hM, r0, am, om, dg, c, pp, hv);
            uint32_t wv = (uint32_t)x;
#pragma unroll
            for (int e = 0; e < kLaneMaxIn; ++e) {
                if (e < kin) {
                    const uint32_t y = (uint32_t)__builtin_amdgcn_ds_bpermute(saddr[e], (int)pp);
                    wv += ((emask >> e) & 1) ? y : 0u;
                }
            }
            uint32_t val = wv - c + kLaneOff;
            u64 Hs = wave_sum_u64(act ? (u64)(uint32_t)x * Rj + hv : 0);
            const u64 Ts = wave_sum_u64(act ? (u64)canon_digit(am, om, dg0) * place_w : 0);
            // Step tables.  T[v][e][j]: change to neuron j when V neuron v fires its
            // e-th canonical rule (-c on j = v, +p on the targets of v).  One
            // odometer step moves the last V neuron that can step up from e to
            // e + 1 and resets every later V neuron from its top digit to 0, so
            // its whole effect is one row per (v, e):
            //   U[v][e] = T[v][e+1] - T[v][e] + sum over later V neurons v' of
            //             (T[v'][0] - T[v'][top]),
            // likewise for the row hash and for the child index (both linear in
            // the digits).  Row r = tbase_v + e: lane r first fetches the rule of
            // row r, then one pass over the rows, last V neuron first, writes the
            // U rows to LDS (lane = neuron) and leaves the hash and child-index
            // changes of row r in lane r.
            int rv = 0, rd = 0, rb = 0, rw = 0;  // lane r < nt: V neuron, canonical digit, its first row, kappa
            for (u64 vq = vmask; vq; vq &= vq - 1) {
                const int v = __builtin_ctzll(vq);
                const int b = __builtin_amdgcn_readlane(tbase, v);
                const int w = __builtin_amdgcn_readlane(kp, v);
                const bool own = lane >= b && lane < b + w;
                rv = own ? v : rv;
                rd = own ? lane - b : rd;
                rb = own ? b : rb;
                rw = own ? w : rw;
            }
            // (shuffles run on every lane: a source lane must not be masked off)
            const bool isrow = lane < nt;
            const uint32_t amr = (uint32_t)__shfl((int)am, rv);
            const int omr = __shfl(om, rv);
            const int r0r = __shfl(r0, rv);
            const u64 plr = __shfl(place_w, rv);
            const int dr = canon_digit(amr, omr, rd);
            const int kr = isrow ? r0r + nth_bit(amr & 0xFFFFu, dr) : 0;
            const int4 Rr = l_rules[kr];
            const u64 hr = isrow ? l_hM[kr] : 0;
            const u64 tr = isrow ? (u64)dr * plr : 0;
            // hash and child-index rows, lane-parallel: row r (not a top digit)
            // takes x[r+1] - x[r] plus, over the later V neurons, x[0] - x[top];
            // those sums are suffix sums over the rows from the next neuron's first
            const int rtop = max(rb + rw - 1, 0);
            const u64 htop = __shfl(hr, rtop), hnext = __shfl(hr, min(lane + 1, 63));
            const u64 ttop = __shfl(tr, rtop), tnext = __shfl(tr, min(lane + 1, 63));
            const u64 e1 = isrow && rd == 0 ? hr - htop : 0;
            const u64 f1 = isrow && rd == 0 ? tr - ttop : 0;
            // suffix sums (rows r .. 63) as total - prefix + own term
            const u64 ph = wave_incl_u64(e1);
            const u64 pt = wave_incl_u64(f1);
            const u64 eh = readlane64(ph, 63) - ph + e1;
            const u64 et = readlane64(pt, 63) - pt + f1;
            const int nxt = rb + rw;  // <= nt <= 32: rows from there on sum to the later neurons'
            const u64 hU = hnext - hr + __shfl(eh, nxt);
            const u64 tU = tnext - tr + __shfl(et, nxt);
            // the U rows, lane = neuron j, rows from the last down (later V
            // neurons first): Sv sums T[v'][0] - T[v'][top] over the later ones
            const int rflag = (rd == rw - 1 ? 1 : 0) | (rd == 0 ? 2 : 0);
            {
                uint32_t Sv = 0, Tprev = 0, Ttop = 0;
                for (int r = nt - 1; r >= 0; --r) {
                    const int v = __builtin_amdgcn_readlane(rv, r);
                    const uint32_t cr = (uint32_t)__builtin_amdgcn_readlane(Rr.z, r);
                    const uint32_t pr = (uint32_t)__builtin_amdgcn_readlane(Rr.w, r);
                    const int fl = __builtin_amdgcn_readlane(rflag, r);
                    const uint32_t Tr = (lane == v ? 0u - cr : 0u) + (((inmask >> v) & 1) ? pr : 0u);
                    if (fl & 1) Ttop = Tr;  // top digit: never steps up
                    else l_tab[r * 64 + lane] = Tprev - Tr + Sv;
                    if (fl & 2) Sv += Tr - Ttop;
                    Tprev = Tr;
                }
            }
            wave_lds_sync();
            // the reference child's canonical digits over V as one mixed-radix
            // number (the last V neuron lowest); it stays below the product of
            // kappa over V (< 2^17 for tables of at most 32 rows) for the whole
            // segment
            uint32_t x0 = 0;
            for (u64 vq = vmask; vq; vq &= vq - 1) {
                const int v = __builtin_ctzll(vq);
                x0 = x0 * (uint32_t)__builtin_amdgcn_readlane(kp, v) + (uint32_t)__builtin_amdgcn_readlane(dg0, v);
            }
            u64 Hc = uni64(Hs);  // hash of the chunk's first child
            u64 Tc = uni64(Ts);  // its child index
            int rowc = 0;        // step row into the chunk's first child (chunks after the first)
            len = __builtin_amdgcn_readfirstlane(len);
            T* srow = stage + (b0 + k) * (long long)m + lane;
            for (int c0 = 0; c0 < len; c0 += 64) {
                const int nch = min(64, len - c0);
                // lane l: the odometer step from child c0 + l to c0 + l + 1, found
                // from the digits of its V value (the lowest digit below its top
                // steps up; U row tbase + digit of that neuron)
                const bool step = c0 + lane + 1 < len;
                uint32_t y = x0 + (uint32_t)(c0 + lane);
                int row = 0;
                bool carry = true;
                for (u64 vq = vmask; vq && __any(carry && step);) {
                    const int v = 63 - __clzll((long long)vq);  // lowest digit first
                    vq &= ~(1ULL << v);
                    const uint32_t w = (uint32_t)__builtin_amdgcn_readlane(kp, v);
                    const int bv = __builtin_amdgcn_readlane(tbase, v);
                    const uint32_t q = udiv_small(y, w);
                    const uint32_t dgt = y - q * w;
                    const bool here = carry && dgt != w - 1;
                    row = here ? bv + (int)dgt : row;
                    carry = carry && !here;
                    y = q;
                }
                // hash and child index of child c0 + l: the chunk's first child's
                // plus the changes of the steps of lanes before l
                const u64 hrow = __shfl(hU, row);
                const u64 trow = __shfl(tU, row);
                const u64 hstep = step ? hrow : 0;
                const u64 tstep = step ? trow : 0;
                const u64 hin = wave_incl_u64(hstep);
                const u64 tin = wave_incl_u64(tstep);
                const bool mine = lane < nch;
                const long long bq = b0 + k + c0 + lane;
                const u64 key = fmix64(Hc + (hin - hstep)) & a.hash_mask;
                // visited-set probe of child bq: the CAS on its home slot is
                // issued here and its answer read after the rows are written
                const bool probe = mine && a.table != nullptr;
                const u64 me = ((key >> 32) << 32) | (u64)(kStageBase + (uint32_t)bq);
                u64 psl = key & a.slot_mask;
                u64 first = kEmpty;
                if (mine) {
                    a.hash[bq] = key;
                    a.cpar[bq] = (int)p;
                    a.ct[bq] = Tc + (tin - tstep);
                    if (probe) first = atomicCAS(&a.table[psl], kEmpty, me);
                }
                Hc += readlane64(hin, 63);
                Tc += readlane64(tin, 63);
                // the rows, one child after the other: one table row per step,
                // read one child ahead
                uint32_t uv = c0 > 0 ? l_tab[rowc * 64 + lane] : 0u;
                for (int l = 0; l < nch; ++l) {
                    val += uv;
                    if (l + 1 < nch) uv = l_tab[__builtin_amdgcn_readlane(row, l) * 64 + lane];
                    if (act) {
                        *srow = (T)(val - kLaneOff);
                        vmin = min(vmin, val);
                        vmax = max(vmax, val);
                    }
                    srow += m;
                }
                rowc = __builtin_amdgcn_readlane(row, 63);
                // finish the probes: the first empty slot taken, or the first
                // entry with the child's tag (queued for a row compare)
                bool queue = false;
                if (probe) {
                    const uint32_t tag = (uint32_t)(key >> 32);
                    u64 e = first;
                    bool placed = false;
                    for (u64 it = 0;;) {
                        if (e == kEmpty) {  // this child's CAS on slot psl succeeded
                            placed = true;
                            break;
                        }
                        if (e != kTomb && (uint32_t)(e >> 32) == tag) {
                            queue = placed = true;
                            break;
                        }
                        if (++it > a.slot_mask) break;
                        psl = (psl + 1) & a.slot_mask;
                        e = __hip_atomic_load(&a.table[psl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (e == kEmpty) e = atomicCAS(&a.table[psl], kEmpty, me);
                    }
                    a.slot[bq] = placed ? (uint32_t)psl : 0u;
                    if (!placed) atomicOr((unsigned long long*)&a.ctr->probe_fail, 1ULL);
                }
                const u64 qm = __ballot(queue);
                if (qm) {
                    u64 qbase = 0;
                    if (lane == 0) qbase = atomicAdd((unsigned long long*)&a.ctr->ncand, (u64)__popcll(qm));
                    qbase = __shfl(qbase, 0);
                    if (queue) a.cand[qbase + __popcll(qm & ((1ULL << lane) - 1))] = (uint32_t)bq;
                }
            }
            k += len;
            u += (u64)len;
            if (k >= cnt) break;
            if (u >= psi_p) {
                // next parent with canonical children
                u64 nb = __ballot(pw > 0 && lane > cur);
                while (nb == 0) {
                    pbase += 64;
                    if (pbase >= n) break;
                    pw = a.psi[min(pbase + lane, n - 1)];
                    if (pbase + lane >= n) pw = 0;
                    cur = -1;
                    nb = __ballot(pw > 0);
                }
                if (nb == 0) break;  // unreachable while g0 + B <= sum of Psi
                cur = __builtin_ctzll(nb);
                p = pbase + cur;
                psi_p = uni64(__shfl(pw, cur));
                u = 0;
                if (p == pf_p) x = pf_x;
                else x = (int)F[p * (long long)m + jl];
                settle(x);
                const u64 nb2 = __ballot(pw > 0 && lane > cur);
                pf_p = -1;
                if (nb2) {
                    pf_p = pbase + __builtin_ctzll(nb2);
                    pf_x = (int)F[pf_p * (long long)m + jl];
                }
                am = neuron_applicable(x, r0, r1, l_rules, om);
                kp = kappa_of(am, om);
                place_w = wave_after_prod64((u64)max(1, om));
            }
            wave_lds_sync();  // the tables are rebuilt for the next segment
        }
    }
    const bool ovf = vmin < kLaneOff || vmax > hi_ok;
    if (__any(ovf) && lane == 0) atomicOr((unsigned long long*)&a.ctr->overflow, 1ULL);
}

hipError_t launch_expand_sparse(int elem_bytes, const DevSystem& s, const ChunkArgs& a, hipStream_t st,
                                bool* probed) {
    *probed = false;
    if (a.B <= 0) return hipSuccess;
    if (s.track < 0 && !s.dlink && s.m <= 64 && s.max_in <= kLaneMaxIn && (size_t)s.r * 24 <= 24 * 1024) {
        *probed = a.table != nullptr;
        // one generation of resident waves (the LDS tables allow 16 per CU);
        // runs of 4 to 4096 children are handed out on the device, where the
        // chunk's true size is known
        const long long waves = std::min<long long>((a.B + 3) / 4, 4096);
        const unsigned blocks = (unsigned)((waves + 3) / 4);
        const size_t lds = (size_t)std::max(1, s.r) * 24 + 4 * (size_t)(kLaneTab * 64) * 4;
        if (elem_bytes == 4) hipLaunchKernelGGL((k_expand_lane<int32_t>), dim3(blocks), dim3(256), lds, st, s, a);
        else hipLaunchKernelGGL((k_expand_lane<uint16_t>), dim3(blocks), dim3(256), lds, st, s, a);
        return hipGetLastError();
    }
    const bool delay = s.dlink != nullptr;
    const int stride = sparse_wave_stride(s.m, delay);
    if ((size_t)stride > 64 * 1024) return hipErrorInvalidValue;  // m too large for this form
    const size_t tbl = table_lds_bytes(s, s.nnz_in);
    const bool tbl_lds = tbl <= (size_t)kTableLdsLimit;
    int wpb = 4;
    while (wpb > 1 && (size_t)wpb * stride + (tbl_lds ? tbl : 0) > 64 * 1024) wpb >>= 1;
    if (tbl_lds && (size_t)wpb * stride + tbl > 64 * 1024) return hipErrorInvalidValue;
    // runs short enough that the chunk spreads over the whole GPU
    int run = 4;
    while (run < 32 && (long long)run * 2 * 8192 <= a.B) run <<= 1;
    if (a.run > 0) run = std::min(a.run, 1024);
    const long long waves = (a.B + run - 1) / run;
    const unsigned blocks = (unsigned)((waves + wpb - 1) / wpb);
    const size_t lds = (size_t)wpb * stride + (tbl_lds ? tbl : 0);
    const dim3 grid(blocks), block(64 * wpb);
#define SNP_SPARSE(T_, L_, D_) hipLaunchKernelGGL((k_expand_sparse<T_, L_, D_>), grid, block, lds, st, s, a, run, stride)
    if (elem_bytes == 4) {
        if (delay) {
            if (tbl_lds) SNP_SPARSE(int32_t, true, true);
            else SNP_SPARSE(int32_t, false, true);
        } else {
            if (tbl_lds) SNP_SPARSE(int32_t, true, false);
            else SNP_SPARSE(int32_t, false, false);
        }
    } else {
        if (delay) {
            if (tbl_lds) SNP_SPARSE(uint16_t, true, true);
            else SNP_SPARSE(uint16_t, false, true);
        } else {
            if (tbl_lds) SNP_SPARSE(uint16_t, true, false);
            else SNP_SPARSE(uint16_t, false, false);
        }
    }
#undef SNP_SPARSE
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Visited set.  Open addressing with linear probing over 64-bit entries
// (tag:32 | ref:32), in two passes:
//   A (a thread per child): probe from the hash slot; claim the first empty
//     slot with a CAS, or stop at the first entry with the child's tag and
//     queue the child for a row compare.
//   B (a wave per queued child): compare the two rows with all 64 lanes; if
//     equal and the entry names a later child of the current chunk, lower it
//     with atomicMin (the entry ends at the first occurrence in canonical
//     order); if different, keep probing (lane 0 drives, compares stay
//     cooperative) until an empty slot or an equal row.
// A keys-first pass (TableArgs::direct) has no rows yet: pass A takes the
// entry with the child's tag as the child's configuration and lowers an entry
// of the chunk to the earliest child with atomicMin at once; k_verify_rows
// checks those rows after the row pass.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ const T* entry_row(const TableArgs& a, uint32_t ref, int m) {
    return ref < kStageBase ? (const T*)a.arena + (u64)ref * (u64)m
                            : (const T*)a.stage + (u64)(ref - kStageBase) * (u64)m;
}

template <typename T>
__global__ __launch_bounds__(256) void k_insert_probe(int m, TableArgs a) {
    const long long b = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long Beff = (long long)a.ctr->beff;
    bool queue = false;
    if (b < Beff) {
        const u64 h = a.hash[b];
        const uint32_t tag = (uint32_t)(h >> 32);
        const u64 mine = ((u64)tag << 32) | (kStageBase + (uint32_t)b);
        u64 sl = h & a.slot_mask;
        bool placed = false;
        for (u64 it = 0; it <= a.slot_mask; ++it) {
            u64 e = __hip_atomic_load(&a.table[sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (e == kEmpty) {
                const u64 old = atomicCAS(&a.table[sl], kEmpty, mine);
                if (old == kEmpty) {
                    placed = true;
                    break;
                }
                e = old;
            }
            if (e != kTomb && (uint32_t)(e >> 32) == tag) {
                // (an entry of the row store has a smaller reference than any child)
                if (a.direct) {
                    if (mine < e) atomicMin(&a.table[sl], mine);
                } else {
                    queue = true;
                }
                placed = true;
                break;
            }
            sl = (sl + 1) & a.slot_mask;
        }
        a.slot[b] = placed ? (uint32_t)sl : 0u;
        if (!placed) atomicOr((unsigned long long*)&a.ctr->probe_fail, 1ULL);
    }
    // append the queued children, one atomic per wave
    const u64 qm = __ballot(queue);
    if (qm) {
        const int lane = threadIdx.x & 63;
        u64 base = 0;
        if (lane == 0) base = atomicAdd(&a.ctr->ncand, (u64)__popcll(qm));
        base = __shfl(base, 0);
        if (queue) a.cand[base + __popcll(qm & ((1ULL << lane) - 1))] = (uint32_t)b;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_insert_compare(int m, TableArgs a) {
    const int lane = threadIdx.x & 63;
    const long long waves = (long long)gridDim.x * (blockDim.x >> 6);
    const long long ncand = (long long)a.ctr->ncand;
    for (long long q = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); q < ncand; q += waves) {
        const long long b = a.cand[q];
        const T* row = (const T*)a.stage + b * (long long)m;
        const u64 h = a.hash[b];
        const uint32_t tag = (uint32_t)(h >> 32);
        const uint32_t myref = kStageBase + (uint32_t)b;
        const u64 mine = ((u64)tag << 32) | myref;
        u64 sl = a.slot[b];
        bool done = false;
        for (u64 it = 0; it <= a.slot_mask && !done; ++it) {
            u64 e = uni64(__hip_atomic_load(&a.table[sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            if (e == kEmpty) {
                u64 old = 0;
                if (lane == 0) old = atomicCAS(&a.table[sl], kEmpty, mine);
                old = uni64(__shfl(old, 0));
                if (old == kEmpty) {
                    done = true;
                    break;
                }
                e = old;
            }
            if (e != kTomb && (uint32_t)(e >> 32) == tag) {
                const uint32_t ref = (uint32_t)e;
                const T* other = entry_row<T>(a, ref, m);
                bool diff = false;
                for (int j = lane; j < m; j += 64) diff |= (row[j] != other[j]);
                if (!__any(diff)) {
                    if (lane == 0 && ref >= kStageBase && myref < ref) atomicMin(&a.table[sl], mine);
                    done = true;
                    break;
                }
                if (lane == 0) atomicAdd((unsigned long long*)&a.ctr->collisions, 1ULL);
            }
            sl = (sl + 1) & a.slot_mask;
        }
        if (lane == 0) {
            a.slot[b] = done ? (uint32_t)sl : 0u;
            if (!done) atomicOr((unsigned long long*)&a.ctr->probe_fail, 1ULL);
        }
    }
}

hipError_t launch_insert(int elem_bytes, int m, const TableArgs& a, hipStream_t st, bool probe) {
    if (a.B <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((a.B + 255) / 256);
    // compare pass: enough waves to cover the device, each looping over the queue
    const unsigned cblocks = (unsigned)std::min<long long>((a.B + 3) / 4, 4096);
    if (elem_bytes == 4) {
        if (probe) hipLaunchKernelGGL(k_insert_probe<int32_t>, dim3(blocks), dim3(256), 0, st, m, a);
        if (!a.direct) hipLaunchKernelGGL(k_insert_compare<int32_t>, dim3(cblocks), dim3(256), 0, st, m, a);
    } else {
        if (probe) hipLaunchKernelGGL(k_insert_probe<uint16_t>, dim3(blocks), dim3(256), 0, st, m, a);
        if (!a.direct) hipLaunchKernelGGL(k_insert_compare<uint16_t>, dim3(cblocks), dim3(256), 0, st, m, a);
    }
    return hipGetLastError();
}

// Up to this many scan tiles, every commit block sums the tile counts before
// its own tile itself (one wave, a few loads each), so the flags need no
// separate scan of tile sums.
constexpr long long kCommitTiles = 1024;

// New-child flags of a chunk: flag[b] = 1 when child b is enumerated
// (b < beff) and owns its visited-set entry.  Within each tile of kScanTile
// children, pos[b] = flags before b and tile_sums[tile] = all flags of the
// tile.
__global__ __launch_bounds__(256) void k_flag_tiles(const u64* __restrict__ table, const uint32_t* __restrict__ slot,
                                                    long long B, const DevCounters* __restrict__ ctr,
                                                    uint32_t* __restrict__ flag, uint32_t* __restrict__ pos,
                                                    uint32_t* __restrict__ tile_sums) {
    __shared__ uint32_t wsum[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const long long beff = min(B, (long long)ctr->beff);
    const long long base = (long long)blockIdx.x * kScanTile + threadIdx.x * 4;
    uint32_t f[4], loc[4], run = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const long long b = base + i;
        f[i] = (b < beff && (uint32_t)table[slot[b]] == kStageBase + (uint32_t)b) ? 1u : 0u;
        loc[i] = run;
        run += f[i];
    }
    uint32_t incl = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    uint32_t tpre = incl - run;
    for (int w = 0; w < wid; ++w) tpre += wsum[w];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (base + i < B) {
            flag[base + i] = f[i];
            pos[base + i] = tpre + loc[i];
        }
    if (threadIdx.x == 255) tile_sums[blockIdx.x] = tpre + run;
}

hipError_t launch_flags(const u64* table, const uint32_t* slot, long long B, DevCounters* ctr, uint32_t* flag,
                        uint32_t* pos, uint32_t* tile_sums, uint32_t* tile_pre, hipStream_t st, bool scan) {
    if (B <= 0) return hipSuccess;
    const long long nt = scan_tiles(B);
    hipLaunchKernelGGL(k_flag_tiles, dim3((unsigned)nt), dim3(256), 0, st, table, slot, B, ctr, flag, pos,
                       tile_sums);
    if (scan || nt > kCommitTiles)  // the commit reads the tile prefix (and the host the total) from here
        hipLaunchKernelGGL((k_scan_sums<uint32_t, false>), dim3(1), dim3(1024), 0, st, tile_sums, tile_pre, nt,
                           (u64*)&ctr->total, nullptr, nullptr);
    return hipGetLastError();
}

// Row copies of the commit stream through the caches: the staged row is read
// once and the stored one is not read again before the next level.
template <typename U>
__device__ __forceinline__ U stream_load(const U* p) {
    if constexpr (sizeof(U) == 16) {
        typedef unsigned int v4u __attribute__((ext_vector_type(4)));
        const v4u v = __builtin_nontemporal_load((const v4u*)p);
        U r;
        __builtin_memcpy(&r, &v, 16);
        return r;
    } else {
        return __builtin_nontemporal_load(p);
    }
}

template <typename U>
__device__ __forceinline__ void stream_store(U* p, const U& x) {
    if constexpr (sizeof(U) == 16) {
        typedef unsigned int v4u __attribute__((ext_vector_type(4)));
        v4u v;
        __builtin_memcpy(&v, &x, 16);
        __builtin_nontemporal_store(v, (v4u*)p);
    } else {
        __builtin_nontemporal_store(x, p);
    }
}

// Commit the new children of a chunk in canonical order: rows below the
// level's limit are copied to the row store and their entries re-pointed at
// it; the rest (past a cap) become tombstones, i.e. are not recorded.  One
// block per 256 children: a thread per child updates the visited set, then the
// block copies the tile's new rows, which land contiguously, in units of U.
template <typename U>
__global__ __launch_bounds__(256) void k_commit(int upr /* units per row */, CommitArgs a) {
    __shared__ int srcb[256];
    __shared__ uint32_t s_pre;
    __shared__ int s_cap_par;
    const long long b0 = (long long)blockIdx.x * 256;
    const long long b = b0 + threadIdx.x;
    const long long tile = b0 / kScanTile;
    if (threadIdx.x == 64) s_cap_par = -1;
    if (threadIdx.x < 64) {
        // new children of the chunk before this block's tile; block 0 also
        // records the chunk's total
        uint32_t pre;
        if (a.tile_pre) {
            pre = a.tile_pre[tile];
        } else {
            const long long nt = (a.B + kScanTile - 1) / kScanTile;
            const long long upto = blockIdx.x == 0 ? nt : tile;
            uint32_t sp = 0, sa = 0;
            for (long long q = threadIdx.x; q < upto; q += 64) {
                const uint32_t v = a.tile_sums[q];
                sp += q < tile ? v : 0u;
                sa += v;
            }
            pre = wave_sum_u32(sp);
            if (blockIdx.x == 0) {
                const uint32_t all = wave_sum_u32(sa);
                if (threadIdx.x == 0) a.ctr->total = all;
            }
        }
        if (threadIdx.x == 0) s_pre = pre;
    }
    __syncthreads();
    const uint32_t p0 = s_pre + a.pos[b0];
    bool isnew = false;
    if (b < a.B && a.flag[b]) {
        isnew = true;
        const uint32_t pb = s_pre + a.pos[b];
        srcb[pb - p0] = threadIdx.x;
        const long long local = a.level_count + (long long)pb;
        const uint32_t sl = a.slot[b];
        const uint32_t tag = (uint32_t)(a.hash[b] >> 32);
        if (local < a.limit) {
            const long long A = a.level_base + local;
            a.table[sl] = ((u64)tag << 32) | (uint32_t)A;
            a.row_slot[A] = sl;
            if (a.par_out) a.par_out[a.par_out_base + local] = (long long)a.cpar[b] + a.par_value_base;
            if (a.t_out) a.t_out[a.par_out_base + local] = (long long)a.ct[b];
            if (local == a.limit - 1) {
                a.ctr->cap_g = (u64)b + 1;
                a.ctr->cap_par = (u64)a.cpar[b];
                a.ctr->cap_t = a.ct[b];
                s_cap_par = a.cpar[b];
            }
        } else {
            a.table[sl] = kTomb;
        }
    }
    const int nnew = __syncthreads_count(isnew);
    if (a.hflag && s_cap_par >= 0) {
        // this block filled the cap: halting parents up to the cap child's
        // parent, and all children of the parents before it
        uint32_t c = 0;
        u64 flo = 0, fhi = 0;
        for (int i = threadIdx.x; i <= s_cap_par; i += 256) {
            c += a.hflag[i];
            if (i < s_cap_par) {
                const u64 f = a.psif[i];
                flo += f & 0x7FFFFFFFull;
                fhi += f >> 31;
            }
        }
        c = wave_sum_u32(c);
        flo = wave_sum_u64(flo);
        fhi = wave_sum_u64(fhi);
        if ((threadIdx.x & 63) == 0) {
            if (c) atomicAdd((unsigned long long*)&a.ctr->count, (u64)c);
            if (flo) atomicAdd((unsigned long long*)&a.ctr->capf_lo, flo);
            if (fhi) atomicAdd((unsigned long long*)&a.ctr->capf_hi, fhi);
        }
    }
    const long long first_local = a.level_count + (long long)p0;
    const int ncopy = a.copy ? (int)max(0LL, min((long long)nnew, a.limit - first_local)) : 0;
    const U* __restrict__ src = (const U*)a.stage + b0 * upr;
    U* __restrict__ dst = (U*)a.arena + (a.level_base + first_local) * upr;
    U* __restrict__ dst2 = a.row2 ? (U*)a.row2 + first_local * upr : nullptr;
    if (upr <= 256) {
        // thread t copies unit o of rows i0, i0 + per, ...: row and unit are
        // fixed per thread, so the loop has no division; four rows' loads are
        // in flight before their stores
        const int per = 256 / upr;
        const int i0 = threadIdx.x / upr, o = threadIdx.x - i0 * upr;
        if (i0 < per) {
            int i = i0;
            for (; i + 3 * per < ncopy; i += 4 * per) {
                U x[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) x[k] = stream_load(src + (long long)srcb[i + k * per] * upr + o);
#pragma unroll
                for (int k = 0; k < 4; ++k) stream_store(dst + (long long)(i + k * per) * upr + o, x[k]);
                if (dst2)
#pragma unroll
                    for (int k = 0; k < 4; ++k) dst2[(long long)(i + k * per) * upr + o] = x[k];
            }
            for (; i < ncopy; i += per) {
                const U x = src[(long long)srcb[i] * upr + o];
                dst[(long long)i * upr + o] = x;
                if (dst2) dst2[(long long)i * upr + o] = x;
            }
        }
    } else {
        // rows of more than 256 units: two rows at a time, two units of each
        // per thread, their four loads in flight before the stores
        int i = 0;
        for (; i + 1 < ncopy; i += 2) {
            const long long s0 = (long long)srcb[i] * upr, s1 = (long long)srcb[i + 1] * upr;
            const long long d0 = (long long)i * upr, d1 = d0 + upr;
            for (int o = threadIdx.x; o < upr; o += 512) {
                const bool two = o + 256 < upr;
                const U x0 = src[s0 + o], x1 = src[s1 + o];
                U y0 = x0, y1 = x1;
                if (two) {
                    y0 = src[s0 + o + 256];
                    y1 = src[s1 + o + 256];
                }
                dst[d0 + o] = x0;
                dst[d1 + o] = x1;
                if (two) {
                    dst[d0 + o + 256] = y0;
                    dst[d1 + o + 256] = y1;
                }
                if (dst2) {
                    dst2[d0 + o] = x0;
                    dst2[d1 + o] = x1;
                    if (two) {
                        dst2[d0 + o + 256] = y0;
                        dst2[d1 + o + 256] = y1;
                    }
                }
            }
        }
        for (; i < ncopy; ++i) {
            const long long s0 = (long long)srcb[i] * upr, d0 = (long long)i * upr;
            for (int o = threadIdx.x; o < upr; o += 256) {
                const U x = src[s0 + o];
                dst[d0 + o] = x;
                if (dst2) dst2[d0 + o] = x;
            }
        }
    }
}

// Row check of a keys-first pass.  Every child that is not the first occurrence
// of its key (its entry names another child of the chunk, or a row of the row
// store) had its row written to its stage row by the row pass; it must equal
// the row its entry names: a row-store row, or the first occurrence's row
// where the row pass put it (the row store for a new child within the limit,
// else its stage row).  A wave takes 64 children and compares the rows of its
// repeats with all lanes; any difference sets ctr->verify_fail.
__device__ __forceinline__ long long new_child_dest(const VerifyArgs& a, long long b) {
    if (!a.flag[b]) return -1;
    const long long q = (long long)a.tile_pre[b / kScanTile] + a.pos[b];
    return q < a.limit_new ? a.arena_row + q : -1;
}

template <typename T>
__global__ __launch_bounds__(256) void k_verify_rows(int m, VerifyArgs a) {
    const int lane = threadIdx.x & 63;
    const long long beff = min(a.B, (long long)a.ctr->beff);
    const long long base = ((long long)blockIdx.x * 4 + (threadIdx.x >> 6)) * 64;
    const long long b = base + lane;
    bool rep = false;
    uint32_t ref = 0;
    // (a child after the one that filled the level's limit is not recorded,
    // whatever it repeats: its row was not built)
    // (the flags name the children that own their entry; only the others read it)
    if (b < beff && !a.flag[b] && (long long)a.tile_pre[b / kScanTile] + a.pos[b] < a.limit_new) {
        ref = (uint32_t)a.table[a.slot[b]];
        rep = true;
    }
    u64 rm = __ballot(rep);
    bool bad = false;
    while (rm) {
        const int l = __ffsll((long long)rm) - 1;
        rm &= rm - 1;
        const uint32_t r = (uint32_t)__shfl((int)ref, l);
        const T* mine = (const T*)a.stage + (base + l) * (long long)m;
        const T* other;
        if (r < kStageBase) {
            other = (const T*)a.arena + (long long)r * m;
        } else {
            const long long o = (long long)(r - kStageBase);
            const long long d = new_child_dest(a, o);
            other = d >= 0 ? (const T*)a.arena + d * m : (const T*)a.stage + o * m;
        }
        bool diff = false;
        for (int j = lane; j < m; j += 64) diff |= mine[j] != other[j];
        bad |= __any(diff);
    }
    if (bad && lane == 0) atomicOr((unsigned long long*)&a.ctr->verify_fail, 1ULL);
}

hipError_t launch_verify(int elem_bytes, int m, const VerifyArgs& a, hipStream_t st) {
    if (a.B <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((a.B + 255) / 256);
    if (elem_bytes == 4) hipLaunchKernelGGL(k_verify_rows<int32_t>, dim3(blocks), dim3(256), 0, st, m, a);
    else hipLaunchKernelGGL(k_verify_rows<uint16_t>, dim3(blocks), dim3(256), 0, st, m, a);
    return hipGetLastError();
}

hipError_t launch_commit(int elem_bytes, int m, const CommitArgs& a_in, hipStream_t st) {
    if (a_in.B <= 0) return hipSuccess;
    CommitArgs a = a_in;
    // the blocks sum the tile counts themselves (unless the flags' scan was forced)
    if (scan_tiles(a.B) <= kCommitTiles && a.copy) a.tile_pre = nullptr;
    const size_t rb = (size_t)m * elem_bytes;
    const uintptr_t al = (uintptr_t)a.stage | (uintptr_t)a.arena | (uintptr_t)a.row2;
    const unsigned blocks = (unsigned)((a.B + 255) / 256);
    if (rb % 16 == 0 && al % 16 == 0)
        hipLaunchKernelGGL(k_commit<uint4>, dim3(blocks), dim3(256), 0, st, (int)(rb / 16), a);
    else if (rb % 4 == 0 && al % 4 == 0)
        hipLaunchKernelGGL(k_commit<uint32_t>, dim3(blocks), dim3(256), 0, st, (int)(rb / 4), a);
    else
        hipLaunchKernelGGL(k_commit<uint16_t>, dim3(blocks), dim3(256), 0, st, (int)(rb / 2), a);
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

__global__ __launch_bounds__(256) void k_fill_i32(int* __restrict__ p, long long n, int v) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(int* p, long long n, int v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

// Block k copies row k between its own buffer and the packed buffer.
template <typename T>
__global__ __launch_bounds__(256) void k_pack_rows(void* const* __restrict__ ptrs, const long long* __restrict__ off,
                                                   T* __restrict__ packed, bool to_packed) {
    const int k = blockIdx.x;
    const long long a = off[k], len = off[k + 1] - a;
    T* own = (T*)ptrs[k];
    for (long long j = threadIdx.x; j < len; j += 256) {
        if (to_packed) packed[a + j] = own[j];
        else own[j] = packed[a + j];
    }
}

hipError_t launch_pack_rows(void* const* ptrs, const long long* off, void* packed, int n, int elem_bytes,
                            bool to_packed, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (elem_bytes == 4)
        hipLaunchKernelGGL(k_pack_rows<int32_t>, dim3(n), dim3(256), 0, st, ptrs, off, (int32_t*)packed, to_packed);
    else
        hipLaunchKernelGGL(k_pack_rows<uint16_t>, dim3(n), dim3(256), 0, st, ptrs, off, (uint16_t*)packed, to_packed);
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void k_rows_insert(int m, const u64* R, u64* table, u64 slot_mask, const T* arena,
                                                     long long first, long long count, u64 hash_mask,
                                                     uint32_t* row_slot, DevCounters* ctr) {
    const int lane = threadIdx.x & 63;
    const long long q = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (q >= count) return;
    const long long A = first + q;
    const u64 h = fmix64(row_hash_wave<T>(arena + A * (long long)m, R, m, lane)) & hash_mask;
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

hipError_t launch_rows_insert(int elem_bytes, int m, const u64* R, u64* table, u64 slot_mask, const void* arena,
                              long long first, long long count, u64 hash_mask, uint32_t* row_slot,
                              DevCounters* ctr, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((count + 3) / 4);
    if (elem_bytes == 4)
        hipLaunchKernelGGL(k_rows_insert<int32_t>, dim3(blocks), dim3(256), 0, st, m, R, table, slot_mask,
                           (const int32_t*)arena, first, count, hash_mask, row_slot, ctr);
    else
        hipLaunchKernelGGL(k_rows_insert<uint16_t>, dim3(blocks), dim3(256), 0, st, m, R, table, slot_mask,
                           (const uint16_t*)arena, first, count, hash_mask, row_slot, ctr);
    return hipGetLastError();
}

// The start of a walk in one launch: the visited set holds C0 alone (row 0
// of the row store) and the counters of the walk's first pass are set.  Every block hashes
// C0 (one wave) and fills its share of the table with empty entries, except
// C0's home slot, which takes C0's entry; block 0 also copies C0 to row 0
// (when the row store is elsewhere), records its slot, checks its range and
// writes -1 as C0's parent and child index when those outputs are given.
template <typename T>
__global__ __launch_bounds__(256) void k_start_walk(int m, const u64* __restrict__ R, u64* __restrict__ table,
                                                    u64 slot_mask, const T* __restrict__ c0, T* __restrict__ arena,
                                                    long long count_max, u64 hash_mask,
                                                    uint32_t* __restrict__ row_slot, DevCounters* __restrict__ sc,
                                                    long long* par0, long long* chi0, const int* nrp,
                                                    const int4* rules, const int* dlink, int mcount,
                                                    long long expand_max, u64 psi_cap, int track,
                                                    u64* psi0, u64* psif0, uint8_t* hflag0, u64* off0, u64* Tdev) {
    __shared__ u64 s_slot, s_entry;
    const int lane = threadIdx.x & 63;
    if (threadIdx.x < 64) {
        const u64 h = fmix64(row_hash_wave<T>(c0, R, m, lane)) & hash_mask;
        if (lane == 0) {
            s_slot = h & slot_mask;
            s_entry = (h >> 32) << 32;  // tag, reference row 0
        }
    }
    __syncthreads();
    const u64 home = s_slot, entry = s_entry;
    const u64 nslots = slot_mask + 1;
    for (u64 i = (u64)blockIdx.x * 256 + threadIdx.x; i < nslots; i += (u64)gridDim.x * 256)
        table[i] = i == home ? entry : kEmpty;
    if (blockIdx.x != 0) return;
    bool bad = false;
    for (int j = threadIdx.x; j < m; j += 256) {
        const T x = c0[j];
        if (arena != c0) arena[j] = x;
        const long long v = (long long)x;
        bad |= v < 0 || v > count_max;
    }
    const int nbad = __syncthreads_count(bad);
    // Psi of C0 (the first level's only parent), its halting flag and offset,
    // when asked: the first pass then needs no Psi launch of its own
    PsiPair psi_c0{0, 0};
    bool halt_c0 = false;
    if (psi0 && threadIdx.x < 64)
        psi_c0 = parent_psi<T>(c0, m, nrp, rules, dlink, mcount, expand_max, track, lane, halt_c0);
    if (threadIdx.x == 0) {
        row_slot[0] = (uint32_t)home;
        if (par0) *par0 = -1;
        if (chi0) *chi0 = -1;
        DevCounters z{};
        z.c0_bad = nbad ? 1 : 0;
        if (psi0) {
            const u64 canon = min(psi_c0.canon, psi_cap), full = min(psi_c0.full, psi_cap);
            psi0[0] = canon;
            psif0[0] = full;
            hflag0[0] = halt_c0 ? 1 : 0;
            off0[0] = 0;
            *Tdev = canon;
            z.psi_total = canon;
            z.psif_lo = full & 0x7FFFFFFFull;
            z.psif_hi = full >> 31;
            z.halting = halt_c0 ? 1 : 0;
        }
        *sc = z;
    }
}

hipError_t launch_start_walk(int elem_bytes, int m, const u64* R, u64* table, u64 slot_mask, const void* c0,
                             void* arena, long long count_max, u64 hash_mask, uint32_t* row_slot, DevCounters* sc,
                             long long* par0, long long* chi0, const DevSystem& s, long long expand_max, u64* psi0,
                             u64* psif0, uint8_t* hflag0, u64* off0, u64* Tdev, hipStream_t st) {
    const unsigned blocks = (unsigned)std::min<u64>((slot_mask + 256) / 256, 4096);
    if (elem_bytes == 4)
        hipLaunchKernelGGL(k_start_walk<int32_t>, dim3(blocks), dim3(256), 0, st, m, R, table, slot_mask,
                           (const int32_t*)c0, (int32_t*)arena, count_max, hash_mask, row_slot, sc, par0, chi0,
                           s.nrule_ptr, s.rules, s.dlink, s.mcount, expand_max, s.psi_cap, s.track, psi0, psif0,
                           hflag0, off0, Tdev);
    else
        hipLaunchKernelGGL(k_start_walk<uint16_t>, dim3(blocks), dim3(256), 0, st, m, R, table, slot_mask,
                           (const uint16_t*)c0, (uint16_t*)arena, count_max, hash_mask, row_slot, sc, par0, chi0,
                           s.nrule_ptr, s.rules, s.dlink, s.mcount, expand_max, s.psi_cap, s.track, psi0, psif0,
                           hflag0, off0, Tdev);
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

}  // namespace snp
