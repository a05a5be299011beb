// Expansion on int8 matrix cores (gfx950 v_mfma_i32_16x16x64_i8).
//
// A block expands a tile of 64 consecutive children g.  The tile is cut into
// segments of one parent each; within a segment of children t_a .. t_b only
// the least significant neurons change digit: V = every neuron with omega >= 2
// from the most significant digit where t_a and t_b differ down to the last
// neuron (all less significant digits wrap inside the range).  With the first
// child of the segment as reference,
//
//   child(t) = child(t_a) + D(t) . M_V,
//
// where M_V stacks the rows of M_Pi of the applicable rules of the neurons in
// V and D(t) holds +1 at the rule a neuron of V fires in child t and -1 at the
// rule it fires in child t_a (0 where they agree): a 64 x K int8 matrix times
// a K x m int8 matrix with int32 accumulation, exact because every entry of
// M_Pi fits int8 and K <= 128.  The reference child comes from the sparse
// pull of Equation next-config; the hash of every row follows from linearity,
// H(child(t)) = H(child(t_a)) + D(t) . H(M_V), without reading the row.
// Segments whose V needs more than 64 neurons or 128 rule columns fall back
// to the sparse pull for each of their children.
//
// Children that fire the later of two twin rules (same neuron, same c and p)
// repeat an earlier child of the same parent and are only marked: a segment
// whose fixed digits already pick a later twin is skipped whole, and within a
// segment the digit walk that builds D(t) also tells which rows are twins;
// their rows are not stored and never reach the visited set.
//
// MFMA operand layout (checked on the device): lane l supplies row l % 16 of
// A and column l % 16 of B, with the 16 int8 of lane group l / 16 covering
// K columns 16 * (l / 16) .. + 15; the 16x16 int32 result lands in lane l as
// rows 4 * (l / 16) + i, column l % 16, i = 0..3.
#include "snp_device.hpp"

namespace snp {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kTile = 64;   // children per block
constexpr int kKMax = 128;  // rule columns of V per segment on the MFMA path
constexpr int kVMax = 64;   // neurons in V per segment on the MFMA path
constexpr int kMTStride = kKMax + 16;  // bytes per column of the transposed M_V tile (padding vs bank conflicts)

struct Lds {
    uint8_t* om;   // [m] omega per neuron
    uint8_t* dg;   // [m] digits of the child being computed by the sparse pull
    uint8_t* dgb;  // [m] digits of the last child of the segment
    uint32_t* am;  // [m] applicable-rule mask (<= 16 rules per neuron) | canonical digits << 16
    uint16_t* cp;  // [m] fired (c << 8 | p) of the child being computed
    int8_t* D;     // [kTile][kKMax]
    int8_t* MT;    // [NT][kMTStride]
    int* klist;    // [kKMax] rule of every K column
    int* vlist;    // [kVMax] neurons of V, most significant first
    int* kbase;    // [kVMax] first K column of every neuron of V
    u64* rowh;     // [kTile] H of every row of the tile
    u64* wsum;     // [4]
    u64* misc;     // [0] reference digits of V that pick a later twin, [1] twin rows of the tile
    int* sc;       // scalars: [0] jstar, [1] nv, [2] kvar
};

__host__ __device__ __forceinline__ size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

__host__ __device__ __forceinline__ size_t int8_lds_bytes(int m, int nt) {
    size_t o = align16((size_t)3 * m);
    o += align16((size_t)4 * m) + align16((size_t)2 * m);
    o += (size_t)kTile * kKMax + (size_t)nt * kMTStride;
    o += align16((size_t)kKMax * 4) + (size_t)kVMax * 4 * 2;
    o += (size_t)kTile * 8 + 6 * 8 + 4 * 4;
    return align16(o);
}

__device__ __forceinline__ Lds carve(unsigned char* smem, int m, int nt) {
    Lds L;
    size_t o = 0;
    L.om = smem;
    L.dg = smem + m;
    L.dgb = smem + 2 * m;
    o = align16((size_t)3 * m);
    L.am = (uint32_t*)(smem + o);
    o += align16((size_t)4 * m);
    L.cp = (uint16_t*)(smem + o);
    o += align16((size_t)2 * m);
    L.D = (int8_t*)(smem + o);
    o += (size_t)kTile * kKMax;
    L.MT = (int8_t*)(smem + o);
    o += (size_t)nt * kMTStride;
    L.klist = (int*)(smem + o);
    o += align16((size_t)kKMax * 4);
    L.vlist = (int*)(smem + o);
    o += (size_t)kVMax * 4;
    L.kbase = (int*)(smem + o);
    o += (size_t)kVMax * 4;
    L.rowh = (u64*)(smem + o);
    o += (size_t)kTile * 8;
    L.wsum = (u64*)(smem + o);
    o += 4 * 8;
    L.misc = (u64*)(smem + o);
    o += 2 * 8;
    L.sc = (int*)(smem + o);
    return L;
}

__device__ __forceinline__ int rule_of(const DevSystem& s, const uint32_t* am, int j, int d) {
    return s.nrule_ptr[j] + nth_bit(am[j] & 0xFFFFu, d);
}

__device__ __forceinline__ bool later_twin(const Lds& L, int j, int d) {
    return L.om[j] >= 2 && !((L.am[j] >> (16 + d)) & 1u);
}

// True (in every thread) when the digits in L.dg pick a later twin somewhere.
__device__ __forceinline__ bool block_any_twin(const Lds& L, int m) {
    bool nc = false;
    for (int j = threadIdx.x; j < m; j += blockDim.x) nc |= later_twin(L, j, L.dg[j]);
    return __syncthreads_or(nc);
}

// Block-wide sum of a 64-bit value (256 threads); every thread gets the total.
__device__ __forceinline__ u64 block_sum64(u64 v, u64* wsum) {
    const u64 w = wave_sum_u64(v);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = w;
    __syncthreads();
    const u64 t = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    return t;
}

// The child of parent row P whose digits are in L.dg, by the sparse pull,
// written to out; returns its H (block-wide).
template <typename T>
__device__ __forceinline__ u64 sparse_child(const DevSystem& s, const Lds& L, const T* P, T* out, bool& ovf) {
    const int m = s.m;
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
        uint16_t v = 0;
        if (L.om[j]) {
            const int4 R = s.rules[rule_of(s, L.am, j, L.dg[j])];
            v = (uint16_t)((R.z << 8) | R.w);
        }
        L.cp[j] = v;
    }
    __syncthreads();
    u64 h = 0;
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
        long long v = (long long)P[j] - (long long)(L.cp[j] >> 8);
        const int e1 = s.in_ptr[j + 1];
        int e = s.in_ptr[j];
        // the source indices come from global memory: eight loads in flight
        // before their LDS reads
        for (; e + 8 <= e1; e += 8) {
            int src[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) src[q] = s.in_src[e + q];
#pragma unroll
            for (int q = 0; q < 8; ++q) v += L.cp[src[q]] & 0xFF;
        }
        for (; e < e1; ++e) v += L.cp[s.in_src[e]] & 0xFF;
        ovf |= (v < 0) | (v > s.count_max);
        out[j] = (T)v;
        h += hterm((uint32_t)v, s.R[j]);
    }
    return block_sum64(h, L.wsum);
}

}  // namespace

size_t int8_lds(int m, int nt) { return int8_lds_bytes(m, nt); }

template <typename T, int NT>
__global__ __launch_bounds__(256) void k_expand_int8(DevSystem s, ChunkArgs a, int tiles_per_block) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int m = s.m;
    const long long tile0 = (long long)blockIdx.x * tiles_per_block;
    const u64 tot = *a.Tdev;
    const long long Beff = tot > a.g0 ? (long long)min((u64)a.B, tot - a.g0) : 0;
    if (blockIdx.x == 0 && tid == 0) a.ctr->beff = (u64)Beff;
    if (tile0 * kTile >= Beff) return;  // whole block
    Lds L = carve(smem, m, NT);
    const T* F = (const T*)a.frontier;
    T* stage = (T*)a.stage;
    bool ovf = false;

    // parent of the first tile's first child: 64-ary search over the offsets;
    // later tiles go on from where the previous one stopped
    long long p;
    u64 ta;
    {
        const u64 g = a.g0 + (u64)(tile0 * kTile);
        long long lo = 0, hi = a.n;
        while (hi - lo > 1) {
            const long long step = (hi - lo + 63) / 64;
            const long long idx = lo + (long long)lane * step;
            const bool ok = idx < hi && a.off[idx] <= g;
            const u64 mask = __ballot(ok);
            lo = lo + (long long)(63 - __clzll((long long)mask)) * step;
            hi = min(hi, lo + step);
        }
        p = lo;  // every wave computes the same value
        ta = g - a.off[p];
    }
    // the parent whose applicability is in L.om / L.am (and whose digit
    // place values wave 0 holds): consecutive tiles mostly share it
    long long have_p = -1;
    u64 place = 0;
    uint32_t ntwin = 0;  // twin children of this block's tiles (thread 0)
    u64 nmfma = 0;       // matrix-core instructions of this block (thread 0)
    // children [.., twin_end) of parent twin_p are all twins: a digit of a
    // neuron above the ones that change there picks a later twin rule
    long long twin_p = -1;
    u64 twin_end = 0;

    for (int tt = 0; tt < tiles_per_block; ++tt) {
    const long long b0 = (tile0 + tt) * kTile;
    if (b0 >= Beff) break;
    const int rows = (int)min((long long)kTile, Beff - b0);
    if (tid == 0) L.misc[1] = 0;
    int c = 0;
    while (c < rows) {
        const u64 psi_p = a.psi[p];
        const int len = (int)min((u64)(rows - c), psi_p - ta);
        const int cend = c + len;
        const u64 tb = ta + (u64)(len - 1);
        const T* P = F + p * (long long)m;

        if (p == twin_p && tb < twin_end) {
            // inside a known run of twins: only their parent and child index
            if (tid >= c && tid < cend) {
                a.cpar[b0 + tid] = -1 - (int)p;
                a.ct[b0 + tid] = ta + (u64)(tid - c);
            }
            if (tid == 0) ntwin += (uint32_t)len;
            c = cend;
            ta += (u64)len;
            if (ta >= psi_p) {
                ++p;
                while (p < a.n && a.psi[p] == 0) ++p;
                ta = 0;
            }
            if (c < rows && p >= a.n) break;  // unreachable while g0 + B <= sum of Psi
            continue;
        }

        // 1. applicability of the parent (kept while the parent stays)
        const bool fresh = p != have_p;
        if (fresh) {
            for (int j = tid; j < m; j += blockDim.x) {
                const int x = (int)P[j];
                uint32_t mask = 0;
                int w = 0;
                const int r0 = s.nrule_ptr[j], r1 = s.nrule_ptr[j + 1];
                for (int q = r0; q < r1; ++q)
                    if (rule_applies(x, s.rules[q])) {
                        mask |= 1u << (q - r0);
                        ++w;
                    }
                L.am[j] = mask | (w >= 2 ? canonical_mask(s.rules, r0, mask) << 16 : 0xFFFF0000u);
                L.om[j] = (uint8_t)w;
            }
            have_p = p;
        }
        if (tid == 0) {
            L.sc[0] = m;
            L.sc[3] = m;
        }
        __syncthreads();
        // 2. digits of the first and last child of the segment
        if (wid == 0) {
            if (fresh) place = digit_place(m, lane, L.om);
            decode_digits_at(m, lane, ta, L.om, L.dg, place);
            decode_digits_at(m, lane, tb, L.om, L.dgb, place);
        }
        __syncthreads();
        // 3. most significant differing digit
        int myj = m;
        for (int j = tid; j < m; j += blockDim.x)
            if (L.dg[j] != L.dgb[j]) myj = min(myj, j);
        if (myj < m) atomicMin(&L.sc[0], myj);
        __syncthreads();
        const int jstar = L.sc[0];
        // 4. V (neurons with omega >= 2 from jstar on) and its rule columns;
        //    do the fixed digits (before jstar) pick a later twin?
        bool fixed_nc = false;
        int first_nc = m;  // most significant fixed digit that picks a later twin
        for (int j = tid; j < jstar; j += blockDim.x)
            if (later_twin(L, j, L.dg[j])) {
                fixed_nc = true;
                first_nc = min(first_nc, j);
            }
        if (first_nc < m) atomicMin(&L.sc[3], first_nc);
        if (wid == 0) {
            int nv = 0;
            for (int base = jstar; base < m; base += 64) {
                const int j = base + lane;
                const bool pred = j < m && L.om[j] >= 2;
                const u64 bm = __ballot(pred);
                const int pos = nv + __popcll(bm & ((1ULL << lane) - 1));
                if (pred && pos < kVMax) L.vlist[pos] = j;
                nv += __popcll(bm);
            }
            int w = 0;
            if (lane < min(nv, kVMax)) w = L.om[L.vlist[lane]];
            int incl = w;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(incl, o);
                if (lane >= o) incl += y;
            }
            const int kb = incl - w;
            const int kvar = __shfl(incl, 63);
            bool rnc = false;
            if (lane < min(nv, kVMax)) {
                L.kbase[lane] = kb;
                const int j = L.vlist[lane];
                for (int d = 0; d < w && kb + d < kKMax; ++d) L.klist[kb + d] = rule_of(s, L.am, j, d);
                rnc = later_twin(L, j, L.dg[j]);
            }
            const u64 refnc = __ballot(rnc);
            if (lane == 0) {
                L.sc[1] = nv;
                L.sc[2] = kvar;
                L.misc[0] = refnc;
            }
        }
        const bool seg_twin = __syncthreads_or(fixed_nc);
        const int nv = L.sc[1];
        const int kvar = L.sc[2];
        const bool mfma = nv <= kVMax && kvar <= a.kmax;
        const u64 seg_rows = (len == 64 ? ~0ULL : ((1ULL << len) - 1)) << c;

        T* refrow = stage + (b0 + c) * (long long)m;
        if (seg_twin) {
            // every child of the segment repeats an earlier one, and so does
            // every child up to the next change of digit J = sc[3]: the run
            // ends at (ta / place_J + 1) * place_J, place_J being the product
            // of omega over the neurons after J (saturated)
            if (tid == 0) L.misc[1] |= seg_rows;
            if (wid == 0) {
                const int J = L.sc[3];
                const int Q = (m + 63) >> 6;
                const int owner = J / Q;
                u64 pj = place;  // this lane's block place value, times its neurons after J
                for (int j = J + 1; j < min(m, owner * Q + Q); ++j) pj = sat_mul(pj, (u64)max(1, (int)L.om[j]));
                pj = __shfl(pj, owner);
                const u64 end = pj >= kPsiSat ? kPsiSat : (ta / pj + 1) * pj;
                if (lane == 0) L.wsum[3] = min(end, psi_p);
            }
            __syncthreads();
            twin_p = p;
            twin_end = L.wsum[3];
        } else if (!mfma) {
            // sparse pull for every child of the segment that is not a twin
            for (int rr = c; rr < cend; ++rr) {
                if (rr > c) {
                    __syncthreads();
                    if (wid == 0) decode_digits(m, lane, ta + (u64)(rr - c), L.om, L.dg);
                    __syncthreads();
                }
                if (block_any_twin(L, m)) {
                    if (tid == 0) L.misc[1] |= 1ULL << rr;
                    continue;
                }
                const u64 h = sparse_child<T>(s, L, P, stage + (b0 + rr) * (long long)m, ovf);
                if (tid == 0) L.rowh[rr] = h;
            }
        } else {
            // 5. reference child (first of the segment) by the sparse pull
            const u64 href = sparse_child<T>(s, L, P, refrow, ovf);
            if (tid == 0) L.rowh[c] = href;
            if (len == 1) {
                if (tid == 0 && L.misc[0]) L.misc[1] |= 1ULL << c;
            } else {
                // 6. D rows and row hashes
                for (int q = tid; q < kTile * kKMax / 4; q += blockDim.x) ((int*)L.D)[q] = 0;
                __syncthreads();
                if (wid == 0) {
                    const u64 refnc = L.misc[0];
                    bool tw = false;
                    if (tid > c && tid < cend) {
                        const int row = tid;
                        uint32_t delta = (uint32_t)(row - c);  // < 64: 32-bit arithmetic throughout
                        u64 h = href;
                        int i = nv - 1;
                        for (; i >= 0 && delta != 0; --i) {
                            const int j = L.vlist[i];
                            const uint32_t w = L.om[j];
                            const int d0 = L.dg[j];
                            const uint32_t x = (uint32_t)d0 + delta;
                            const int d1 = (int)(x % w);
                            delta = x / w;
                            tw |= later_twin(L, j, d1);
                            if (d1 != d0) {
                                const int k1 = L.kbase[i] + d1, k0 = L.kbase[i] + d0;
                                L.D[row * kKMax + k1] = 1;
                                L.D[row * kKMax + k0] = -1;
                                h += s.hM[L.klist[k1]] - s.hM[L.klist[k0]];
                            }
                        }
                        // neurons 0 .. i of V keep the reference digits
                        if (i >= 0) tw |= (refnc & ((2ULL << i) - 1)) != 0;
                        L.rowh[row] = h;
                    } else if (tid == c) {
                        tw = refnc != 0;
                    }
                    const u64 bm = __ballot(tw);
                    if (lane == 0) L.misc[1] |= bm;
                }
                const int kpad = (kvar + 63) & ~63;
                // instructions this segment issues: (m / NT) column tiles x 4 waves x
                // (kpad / 64) K steps x 4 row blocks x NT / 64 column blocks
                if (tid == 0) nmfma += (u64)((m + NT - 1) / NT) * 4 * (kpad / 64) * 4 * (NT / 64);
                // 7. column tiles: stage M_V transposed, multiply, add the reference row
                for (int n0 = 0; n0 < m; n0 += NT) {
                    __syncthreads();
                    for (int q = tid; q < kpad * NT; q += blockDim.x) {
                        const int k = q / NT, n = q - k * NT;
                        int8_t v = 0;
                        if (k < kvar && n0 + n < m) v = s.M8[(long long)L.klist[k] * m + n0 + n];
                        L.MT[n * kMTStride + k] = v;
                    }
                    __syncthreads();
                    const u64 twm = L.misc[1];
                    constexpr int CB = NT / 64;  // 16-column blocks per wave
                    v4i acc[4][CB];
#pragma unroll
                    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = v4i{0, 0, 0, 0};
                    const int colw = wid * (NT / 4);
                    for (int ks = 0; ks < kpad; ks += 64) {
                        v4i af[4], bf[CB];
#pragma unroll
                        for (int rb = 0; rb < 4; ++rb)
                            af[rb] = *(const v4i*)&L.D[(16 * rb + (lane & 15)) * kKMax + ks + 16 * (lane >> 4)];
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb)
                            bf[cb] = *(const v4i*)&L.MT[(colw + 16 * cb + (lane & 15)) * kMTStride + ks + 16 * (lane >> 4)];
#pragma unroll
                        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                            for (int cb = 0; cb < CB; ++cb)
                                acc[rb][cb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[rb], bf[cb], acc[rb][cb], 0, 0, 0);
                    }
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) {
                        const int col = n0 + colw + 16 * cb + (lane & 15);
                        if (col >= m) continue;
                        const long long refv = (long long)refrow[col];
#pragma unroll
                        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                const int row = 16 * rb + 4 * (lane >> 4) + i;
                                if (row <= c || row >= cend || ((twm >> row) & 1)) continue;
                                const long long v = refv + acc[rb][cb][i];
                                ovf |= (v < 0) | (v > s.count_max);
                                stage[(b0 + row) * (long long)m + col] = (T)v;
                            }
                    }
                }
            }
        }
        __syncthreads();
        // 8. per-row outputs of the segment; a twin row holds -1 - parent
        if (tid == 0) ntwin += (uint32_t)__popcll(L.misc[1] & seg_rows);
        if (tid >= c && tid < cend) {
            const bool tw = (L.misc[1] >> tid) & 1;
            if (!tw) a.hash[b0 + tid] = fmix64(L.rowh[tid]) & a.hash_mask;
            a.cpar[b0 + tid] = tw ? -1 - (int)p : (int)p;
            a.ct[b0 + tid] = ta + (u64)(tid - c);
        }
        // next segment: the rest of this parent's children, else the next
        // parent with children
        c = cend;
        ta += (u64)len;
        if (ta >= psi_p) {
            ++p;
            while (p < a.n && a.psi[p] == 0) ++p;
            ta = 0;
        }
        __syncthreads();
        if (c < rows && p >= a.n) break;  // unreachable while g0 + B <= sum of Psi
    }
    if (p >= a.n) break;
    }
    if (__syncthreads_or(ovf) && tid == 0) atomicOr((unsigned long long*)&a.ctr->overflow, 1ULL);
    if (tid == 0 && ntwin) atomicAdd((unsigned long long*)&a.ctr->twins, (u64)ntwin);
    if (tid == 0 && nmfma) atomicAdd((unsigned long long*)&a.ctr->mfma, nmfma);
}

hipError_t launch_expand_int8(int elem_bytes, const DevSystem& s, const ChunkArgs& a, hipStream_t st) {
    if (a.B <= 0) return hipSuccess;
    const bool wide = int8_lds_bytes(s.m, 128) <= 64 * 1024;
    const size_t lds = int8_lds_bytes(s.m, wide ? 128 : 64);
    if (lds > 64 * 1024) return hipErrorInvalidValue;
    // consecutive tiles per block (they mostly share a parent, and runs of
    // twins carry over), keeping about four rounds of resident blocks (LDS
    // bounds them: 160 KiB per CU, 256 CUs) for balance
    const long long tiles = (a.B + kTile - 1) / kTile;
    const long long resident = 256LL * std::max<long long>(1, (160 * 1024) / (long long)lds);
    const int tpb = (int)std::max<long long>(1, std::min<long long>(16, tiles / (4 * resident)));
    const unsigned blocks = (unsigned)((tiles + tpb - 1) / tpb);
#define SNP_I8(TT, NN) hipLaunchKernelGGL((k_expand_int8<TT, NN>), dim3(blocks), dim3(256), lds, st, s, a, tpb)
    if (elem_bytes == 4) {
        if (wide) SNP_I8(int32_t, 128);
        else SNP_I8(int32_t, 64);
    } else {
        if (wide) SNP_I8(uint16_t, 128);
        else SNP_I8(uint16_t, 64);
    }
#undef SNP_I8
    return hipGetLastError();
}

}  // namespace snp
