// Expansion on int8 matrix cores (gfx950 v_mfma_i32_16x16x64_i8).
//
// A block expands a tile of 256 consecutive canonical children (children whose
// every digit is canonical: twins, which repeat an earlier child, are never
// enumerated).  The tile is cut into segments of one parent each; within a
// segment of canonical children u_a .. u_b only the least significant
// canonical digits change: V = every neuron with kappa >= 2 (two or more
// canonical digits) from the most significant digit where u_a and u_b differ
// down to the last neuron (all less significant digits wrap inside the
// range).  With the first child of the segment as reference,
//
//   child(u) = child(u_a) + D(u) . M_V,
//
// where M_V stacks the rows of M_Pi of the canonical rules of the neurons in
// V and D(u) holds +1 at the rule a neuron of V fires in child u and -1 at the
// rule it fires in child u_a (0 where they agree): a 256 x K int8 matrix times
// a K x m int8 matrix with int32 accumulation, exact because every entry of
// M_Pi fits int8 and K <= 64.  The reference child comes from the sparse
// pull of Equation next-config; the hash of every row follows from linearity,
// H(child(u)) = H(child(u_a)) + D(u) . H(M_V), without reading the row, and
// so does its child index t (linear in the digits, with the place values of
// the full mixed radix).  A segment whose V needs more than 64 neurons or 64
// rule columns is halved until it fits; a single child is computed by the pull.
// When a segment starts right after the block's previous one in the same
// parent (consecutive tiles of a block mostly do), its reference child is the
// previous segment's last child with the rows of M_Pi of the few neurons whose
// digit changed swapped, instead of a full pull.
// The transposed M_V of a column tile is staged once and serves the segment's
// four 64-row quarters, each a 4 x (NT / 64) grid of 16 x 16 products per wave.
//
// Keys-first passes run the kernel twice.  Mode 1 (keys) computes only every
// child's key, parent and child index: the reference child's H is H(parent)
// plus H(M_k) of the rules it fires, the others follow by linearity as above;
// no row is built.  After the visited-set probe has named the new children,
// mode 2 (rows) builds the rows and writes each new child's row straight to
// its place in the row store, every other row to its stage row (where the row
// check reads it).  Mode 0 writes every row to the stage.
//
// MFMA operand layout (checked on the device): lane l supplies row l % 16 of
// A and column l % 16 of B, with the 16 int8 of lane group l / 16 covering
// K columns 16 * (l / 16) .. + 15; the 16x16 int32 result lands in lane l as
// rows 4 * (l / 16) + i, column l % 16, i = 0..3.
#include "snp_device.hpp"

namespace snp {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kTile = 256;  // children per block tile (one per thread)
constexpr int kKMax = 64;   // rule columns of V per segment on the MFMA path (one 64-deep K step)
constexpr int kVMax = 64;   // neurons in V per segment on the MFMA path
constexpr int kMTStride = kKMax + 16;  // bytes per column of the transposed M_V tile (padding vs bank conflicts)
static_assert(2 * 4608 <= kTile * kKMax, "the pull's fired-rule words fit in D for every m the library takes");
constexpr int kIncMax = 32;  // most changed digits for a reference child derived from the previous segment's last

struct Lds {
    uint8_t* om;   // [m] omega per neuron
    uint8_t* dg;   // [m] canonical digits of the child being computed by the sparse pull
    uint8_t* dgb;  // [m] canonical digits of the last child of the segment
    uint32_t* am;  // [m] applicable-rule mask (<= 16 rules per neuron) | canonical digits << 16
    uint8_t* dp;   // [m] canonical digits of the previous segment's last child
    uint16_t* cp;  // [m] fired (c << 8 | p) of the child being computed by the pull (shares D's
                   // bytes: the pull ends before D is filled)
    int8_t* D;     // [kTile][kKMax]
    int8_t* MT;    // [NT][kMTStride]
    int* klist;    // [kKMax] rule of every K column
    int* vlist;    // [kVMax] neurons of V, most significant first
    int* kbase;    // [kVMax] first K column of every neuron of V
    u64* rowh;     // [kTile] H of every row of the tile
    void** rowdst; // [kTile] mode 2: where every row of the tile goes (shares rowh's bytes: that
                   // mode computes no H)
    u64* placev;   // [kVMax] place value (over omega) of every neuron of V
    u64* wsum;     // [5]: [0..3] block sums, [4] the reference child's index t
    int* sc;       // scalars: [0] jstar, [1] nv, [2] kvar, [3] changed digits
    int* chg;      // [kIncMax] neurons whose digit changed, then their old and new rules
    int* k0;       //   (share D's bytes: used before D is filled)
    int* k1;
};

__host__ __device__ __forceinline__ size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

__host__ __device__ __forceinline__ size_t int8_lds_bytes(int m, int nt) {
    size_t o = align16((size_t)4 * m);
    o += align16((size_t)4 * m);
    o += (size_t)kTile * kKMax + (size_t)nt * kMTStride;
    o += align16((size_t)kKMax * 4) + (size_t)kVMax * 4 * 2;
    o += (size_t)kTile * 8 + (size_t)kVMax * 8 + 5 * 8 + 4 * 4;
    return align16(o);
}

__device__ __forceinline__ Lds carve(unsigned char* smem, int m, int nt) {
    Lds L;
    size_t o = 0;
    L.om = smem;
    L.dg = smem + m;
    L.dgb = smem + 2 * m;
    L.dp = smem + 3 * m;
    o = align16((size_t)4 * m);
    L.am = (uint32_t*)(smem + o);
    o += align16((size_t)4 * m);
    L.D = (int8_t*)(smem + o);
    L.cp = (uint16_t*)L.D;  // 2 m <= kTile * kKMax for every m the library takes
    L.chg = (int*)L.D;
    L.k0 = L.chg + kIncMax;
    L.k1 = L.k0 + kIncMax;
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
    L.rowdst = (void**)L.rowh;
    o += (size_t)kTile * 8;
    L.placev = (u64*)(smem + o);
    o += (size_t)kVMax * 8;
    L.wsum = (u64*)(smem + o);
    o += 5 * 8;
    L.sc = (int*)(smem + o);
    return L;
}

// Rule fired by neuron j at canonical digit e.
__device__ __forceinline__ int rule_of(const DevSystem& s, const Lds& L, int j, int e) {
    return s.nrule_ptr[j] + nth_bit(L.am[j] & 0xFFFFu, canon_digit(L.am[j], L.om[j], e));
}

__device__ __forceinline__ int kappa(const Lds& L, int j) { return kappa_of(L.am[j], L.om[j]); }

// Block-wide sum of a 64-bit value (256 threads); every thread gets the total.
__device__ __forceinline__ u64 block_sum64(u64 v, u64* wsum) {
    const u64 w = wave_sum_u64(v);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = w;
    __syncthreads();
    const u64 t = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    return t;
}

// The child of parent row P whose canonical digits are in L.dg, by the sparse
// pull, written to out; returns its H (block-wide).
template <typename T>
__device__ __forceinline__ u64 sparse_child(const DevSystem& s, const Lds& L, const T* P, T* out, bool& ovf) {
    const int m = s.m;
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
        uint16_t v = 0;
        if (L.om[j]) {
            const int4 R = s.rules[rule_of(s, L, j, L.dg[j])];
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

// The child whose canonical digits are in L.dg from `prev`, the row of the
// child of the same parent whose digits are in L.dp: every neuron j whose
// digit differs (nch of them, listed in L.chg) trades the row of M_Pi of its
// old rule for that of its new one (Equation next-config: the two children
// differ by exactly those rows), read from the int8 copy of M_Pi; the row's H
// follows from H(M_k) the same way.  Written to out; returns H (block-wide).
template <typename T>
__device__ __forceinline__ u64 delta_child(const DevSystem& s, const Lds& L, const T* prev, T* out, u64 hprev,
                                           int nch, bool& ovf) {
    const int m = s.m;
    if ((int)threadIdx.x < nch) {
        const int j = L.chg[threadIdx.x];
        L.k0[threadIdx.x] = rule_of(s, L, j, L.dp[j]);
        L.k1[threadIdx.x] = rule_of(s, L, j, L.dg[j]);
    }
    __syncthreads();
    for (int n = threadIdx.x; n < m; n += blockDim.x) {
        long long v = (long long)prev[n];
        for (int q = 0; q < nch; ++q)
            v += (int)s.M8[(long long)L.k1[q] * m + n] - (int)s.M8[(long long)L.k0[q] * m + n];
        ovf |= (v < 0) | (v > s.count_max);
        out[n] = (T)v;
    }
    u64 h = hprev;
    for (int q = 0; q < nch; ++q) h += s.hM[L.k1[q]] - s.hM[L.k0[q]];
    __syncthreads();  // L.k0 / L.k1 (D's bytes) are read before D is cleared
    return h;
}

}  // namespace

size_t int8_lds(int m, int nt) { return int8_lds_bytes(m, nt); }

template <typename T, int NT, int MODE>
__global__ __launch_bounds__(256) void k_expand_int8(DevSystem s, ChunkArgs a, int tiles_per_block) {
    constexpr bool KEYS = MODE == 1, ROWS = MODE == 2;
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
    const int kmax = min(a.kmax, kKMax);

    // parent of the first tile's first child: 64-ary search over the offsets;
    // later tiles go on from where the previous one stopped
    long long p;
    u64 ua;
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
        ua = g - a.off[p];
    }
    // the parent whose applicability is in L.om / L.am (and whose place values
    // of canonical digits and of child indices wave 0 holds): consecutive
    // tiles mostly share it
    long long have_p = -1;
    u64 place_k = 0, place_w = 0;
    u64 nmfma = 0;  // matrix-core instructions of this block (thread 0)
    u64 my_t = 0;   // thread r: child index t of row r of the tile
    // the block's previous segment: parent, canonical index and row of its
    // last child, and that row's H (its digits are in L.dp)
    long long last_p = -1;
    const T* last_row = nullptr;
    u64 last_u = 0, last_h = 0;
    u64 hP = 0;  // mode 1: H of the parent in L.om / L.am

    for (int tt = 0; tt < tiles_per_block; ++tt) {
    const long long b0 = (tile0 + tt) * kTile;
    if (b0 >= Beff) break;
    const int rows = (int)min((long long)kTile, Beff - b0);
    if constexpr (ROWS) {
        // destinations of the tile's rows (the previous tile's are no longer
        // read).  A child with q new children before it in the chunk and
        // q >= limit_new comes after the child that filled the level's limit:
        // its row is never read (a repeat is of an earlier child), so it is not
        // built; those children end the chunk, so the block stops at the first.
        __syncthreads();
        for (int r = tid; r < kTile; r += blockDim.x) {
            const long long b = b0 + r;
            T* d = nullptr;
            if (b < Beff) {
                const long long q = (long long)a.tile_pre[b / kScanTile] + a.pos[b];
                if (q < a.limit_new)
                    d = a.flag[b] ? (T*)a.arena + (a.arena_row + q) * (long long)m : stage + b * (long long)m;
            }
            L.rowdst[r] = d;
        }
        __syncthreads();
        if (!L.rowdst[0]) break;
    }
    bool past = false;  // mode 2: the rest of the chunk lies past the level's limit
    int c = 0;
    while (c < rows) {
        const u64 psi_p = a.psi[p];
        int len = (int)min((u64)(rows - c), psi_p - ua);
        const T* P = F + p * (long long)m;

        // 1. applicability of the parent (kept while the parent stays)
        const bool fresh = p != have_p;
        if (fresh) {
            for (int j = tid; j < m; j += blockDim.x) {
                int w;
                L.am[j] = neuron_applicable((int)P[j], s.nrule_ptr[j], s.nrule_ptr[j + 1], s.rules, w);
                L.om[j] = (uint8_t)w;
            }
            have_p = p;
            if constexpr (KEYS) {
                u64 hp = 0;
                for (int j = tid; j < m; j += blockDim.x) hp += hterm((uint32_t)P[j], s.R[j]);
                hP = block_sum64(hp, L.wsum);
            }
            __syncthreads();
            if (wid == 0) {
                place_k = canon_place(m, lane, L.om, L.am);
                place_w = digit_place(m, lane, L.om);
            }
        }
        // 2-4. digits of the segment's first and last child, V and its rule
        //      columns; a segment whose V does not fit is halved until it does
        int nv = 0, kvar = 0;
        for (;;) {
            if (tid == 0) L.sc[0] = m;
            const u64 ub = ua + (u64)(len - 1);
            if (wid == 0) {
                canon_decode(m, lane, ua, L.om, L.am, L.dg, place_k);
                canon_decode(m, lane, ub, L.om, L.am, L.dgb, place_k);
            }
            __syncthreads();
            int myj = m;
            for (int j = tid; j < m; j += blockDim.x)
                if (L.dg[j] != L.dgb[j]) myj = min(myj, j);
            if (myj < m) atomicMin(&L.sc[0], myj);
            __syncthreads();
            const int jstar = L.sc[0];
            if (wid == 0) {
                int cnt = 0;
                for (int base = jstar; base < m; base += 64) {
                    const int j = base + lane;
                    const bool pred = j < m && kappa(L, j) >= 2;
                    const u64 bm = __ballot(pred);
                    const int pos = cnt + __popcll(bm & ((1ULL << lane) - 1));
                    if (pred && pos < kVMax) L.vlist[pos] = j;
                    cnt += __popcll(bm);
                }
                const bool inv = lane < min(cnt, kVMax);
                const int jv = inv ? L.vlist[lane] : 0;
                const int w = inv ? kappa(L, jv) : 0;
                int incl = w;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const int y = __shfl_up(incl, o);
                    if (lane >= o) incl += y;
                }
                const int kb = incl - w;
                const int kv = __shfl(incl, 63);
                // place value of neuron jv: its block's (lane jv / Q of place_w)
                // times omega of the block's neurons after it
                const int Q = (m + 63) >> 6;
                const u64 pb = __shfl(place_w, jv / Q);
                if (inv) {
                    L.kbase[lane] = kb;
                    for (int d = 0; d < w && kb + d < kKMax; ++d) L.klist[kb + d] = rule_of(s, L, jv, d);
                    u64 pl = pb;
                    for (int j = jv + 1; j < min(m, (jv / Q) * Q + Q); ++j) pl *= (u64)max(1, (int)L.om[j]);
                    L.placev[lane] = pl;
                }
                const u64 t_ref = child_index(m, lane, L.om, L.am, L.dg, place_w);
                if (lane == 0) {
                    L.sc[1] = cnt;
                    L.sc[2] = kv;
                    L.wsum[4] = t_ref;
                }
            }
            __syncthreads();
            nv = L.sc[1];
            kvar = L.sc[2];
            if (len == 1 || (nv <= kVMax && kvar <= kmax)) break;
            len = (len + 1) / 2;
            __syncthreads();  // L.dg / L.dgb and the scalars are rewritten
        }
        const int cend = c + len;
        if (tid == c) my_t = L.wsum[4];
        if constexpr (ROWS) {
            if (!L.rowdst[c]) {
                past = true;
                break;
            }
        }

        // 5. reference child (first of the segment): from the previous
        //    segment's last child when that is its predecessor in this parent
        //    and few digits differ, else by the sparse pull; mode 1 takes only
        //    its H
        T* refrow = ROWS ? (T*)L.rowdst[c] : stage + (b0 + c) * (long long)m;
        u64 href = 0;
        if constexpr (KEYS) {
            u64 hs = 0;
            for (int j = tid; j < m; j += blockDim.x)
                if (L.om[j]) hs += s.hM[rule_of(s, L, j, L.dg[j])];
            href = hP + block_sum64(hs, L.wsum);
        } else {
            int nch = kIncMax + 1;
            if (p == last_p && ua == last_u + 1) {
                if (tid == 0) L.sc[3] = 0;
                __syncthreads();
                for (int j = tid; j < m; j += blockDim.x)
                    if (L.dg[j] != L.dp[j]) {
                        const int q = atomicAdd(&L.sc[3], 1);
                        if (q < kIncMax) L.chg[q] = j;
                    }
                __syncthreads();
                nch = L.sc[3];
            }
            href = nch <= kIncMax ? delta_child<T>(s, L, last_row, refrow, last_h, nch, ovf)
                                  : sparse_child<T>(s, L, P, refrow, ovf);
        }
        if (!ROWS && tid == 0) L.rowh[c] = href;
        if (len > 1) {
            // 6. D rows, row hashes and child indices (thread r: row r)
            if constexpr (!KEYS)
                for (int q = tid; q < kTile * kKMax / 16; q += blockDim.x) ((int4*)L.D)[q] = make_int4(0, 0, 0, 0);
            const u64 t_c = L.wsum[4];
            __syncthreads();
            if (tid > c && tid < cend) {
                const int row = tid;
                uint32_t delta = (uint32_t)(row - c);  // < 256: 32-bit arithmetic throughout
                u64 h = href, tr = t_c;
                for (int i = nv - 1; i >= 0 && delta != 0; --i) {
                    const int j = L.vlist[i];
                    const uint32_t w = (uint32_t)kappa(L, j);
                    const int e0 = L.dg[j];
                    const uint32_t x = (uint32_t)e0 + delta;
                    const int e1 = (int)(x % w);
                    delta = x / w;
                    if (e1 != e0) {
                        const int k1 = L.kbase[i] + e1, k0 = L.kbase[i] + e0;
                        if constexpr (!KEYS) {
                            L.D[row * kKMax + k1] = 1;
                            L.D[row * kKMax + k0] = -1;
                        }
                        if constexpr (!ROWS) {
                            h += s.hM[L.klist[k1]] - s.hM[L.klist[k0]];
                            const int om = L.om[j];
                            tr += (u64)(long long)(canon_digit(L.am[j], om, e1) - canon_digit(L.am[j], om, e0)) *
                                  L.placev[i];
                        }
                    }
                }
                if constexpr (!ROWS) {
                    L.rowh[row] = h;
                    my_t = tr;
                }
            }
            if constexpr (!KEYS) {
                // quarters of 64 rows that hold rows c + 1 .. cend - 1
                const int q0 = (c + 1) >> 6, q1 = (cend - 1) >> 6;
                // instructions this segment issues: (m / NT) column tiles x 4 waves x
                // quarters x 4 row blocks x NT / 64 column blocks
                if (tid == 0) nmfma += (u64)((m + NT - 1) / NT) * 4 * (q1 - q0 + 1) * 4 * (NT / 64);
                // 7. column tiles: stage M_V transposed, then every quarter's product
                //    plus the reference row.  Only the kvar live rule columns are
                //    staged: D is 0 in every later column, so whatever MT holds there
                //    adds nothing.  With m a multiple of 16 a rule's slice of the tile
                //    is read as 16-byte vectors.
                for (int n0 = 0; n0 < m; n0 += NT) {
                    __syncthreads();
                    if ((m & 15) == 0) {
                        constexpr int G = NT / 16;
                        for (int q = tid; q < kvar * G; q += blockDim.x) {
                            const int k = q / G, n = 16 * (q - k * G);
                            if (n0 + n >= m) continue;
                            const int4 v = *(const int4*)&s.M8[(long long)L.klist[k] * m + n0 + n];
                            const int8_t* b = (const int8_t*)&v;
#pragma unroll
                            for (int i = 0; i < 16; ++i) L.MT[(n + i) * kMTStride + k] = b[i];
                        }
                    } else {
                        for (int q = tid; q < kvar * NT; q += blockDim.x) {
                            const int k = q / NT, n = q - k * NT;
                            if (n0 + n < m) L.MT[n * kMTStride + k] = s.M8[(long long)L.klist[k] * m + n0 + n];
                        }
                    }
                    __syncthreads();
                    // The product is taken transposed, (D . M_V)^T = M_V^T . D^T: the
                    // staged MT is the A operand and the D rows the B operand, so lane
                    // l ends with child row l % 16 of its 16-row block at the four
                    // consecutive columns 4 (l / 16) .. + 3 of each 16-column block,
                    // stored as one vector.
                    constexpr int CB = NT / 64;  // 16-column blocks per wave
                    const int colw = wid * (NT / 4);
                    const bool vec = (m & 3) == 0;  // rows and 4-column groups aligned for vector access
                    v4i af[CB];
                    int refv[CB][4];
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) {
                        af[cb] = *(const v4i*)&L.MT[(colw + 16 * cb + (lane & 15)) * kMTStride + 16 * (lane >> 4)];
                        const int col0 = n0 + colw + 16 * cb + 4 * (lane >> 4);
#pragma unroll
                        for (int i = 0; i < 4; ++i) refv[cb][i] = col0 + i < m ? (int)refrow[col0 + i] : 0;
                    }
                    for (int qr = q0; qr <= q1; ++qr) {
#pragma unroll
                        for (int rb = 0; rb < 4; ++rb) {
                            const int row = 64 * qr + 16 * rb + (lane & 15);
                            const v4i bf = *(const v4i*)&L.D[row * kKMax + 16 * (lane >> 4)];
                            v4i acc[CB];
#pragma unroll
                            for (int cb = 0; cb < CB; ++cb)
                                acc[cb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[cb], bf, v4i{0, 0, 0, 0}, 0, 0, 0);
                            if (row <= c || row >= cend) continue;
                            T* out = ROWS ? (T*)L.rowdst[row] : stage + (b0 + row) * (long long)m;
                            if (ROWS && !out) continue;
                            if constexpr (sizeof(T) == 2 && CB % 2 == 0) {
                                // 16-bit rows: lanes l and l ^ 16 (column groups g, g ^ 1 of one
                                // row) trade one block's four counts, so every lane stores eight
                                // consecutive columns (16 bytes) of block cb0 (g even) or cb1 (g odd)
                                if ((m & 7) == 0 && n0 + colw + 16 * CB <= m) {
                                    const int g = lane >> 4;
#pragma unroll
                                    for (int cb0 = 0; cb0 < CB; cb0 += 2) {
                                        uint32_t pk[2][2];
#pragma unroll
                                        for (int h = 0; h < 2; ++h) {
                                            const int cb = cb0 + h;
                                            long long v[4];
#pragma unroll
                                            for (int i = 0; i < 4; ++i) {
                                                v[i] = (long long)refv[cb][i] + acc[cb][i];
                                                ovf |= (v[i] < 0) | (v[i] > s.count_max);
                                            }
                                            pk[h][0] = (uint32_t)(uint16_t)v[0] | ((uint32_t)(uint16_t)v[1] << 16);
                                            pk[h][1] = (uint32_t)(uint16_t)v[2] | ((uint32_t)(uint16_t)v[3] << 16);
                                        }
                                        const bool even = (g & 1) == 0;
                                        const uint32_t r0 = (uint32_t)__shfl_xor((int)(even ? pk[1][0] : pk[0][0]), 16);
                                        const uint32_t r1 = (uint32_t)__shfl_xor((int)(even ? pk[1][1] : pk[0][1]), 16);
                                        const int col = even ? n0 + colw + 16 * cb0 + 4 * g
                                                             : n0 + colw + 16 * (cb0 + 1) + 4 * (g - 1);
                                        const uint4 w = even ? make_uint4(pk[0][0], pk[0][1], r0, r1)
                                                             : make_uint4(r0, r1, pk[1][0], pk[1][1]);
                                        *(uint4*)(out + col) = w;
                                    }
                                    continue;
                                }
                            }
#pragma unroll
                            for (int cb = 0; cb < CB; ++cb) {
                                const int col0 = n0 + colw + 16 * cb + 4 * (lane >> 4);
                                long long v[4];
#pragma unroll
                                for (int i = 0; i < 4; ++i) {
                                    v[i] = (long long)refv[cb][i] + acc[cb][i];
                                    ovf |= (col0 + i < m) & ((v[i] < 0) | (v[i] > s.count_max));
                                }
                                if (vec && col0 + 3 < m) {
                                    if constexpr (sizeof(T) == 4) {
                                        *(int4*)(out + col0) = make_int4((int)v[0], (int)v[1], (int)v[2], (int)v[3]);
                                    } else {
                                        const uint2 pk = make_uint2((uint32_t)(uint16_t)v[0] | ((uint32_t)(uint16_t)v[1] << 16),
                                                                    (uint32_t)(uint16_t)v[2] | ((uint32_t)(uint16_t)v[3] << 16));
                                        *(uint2*)(out + col0) = pk;
                                    }
                                } else {
#pragma unroll
                                    for (int i = 0; i < 4; ++i)
                                        if (col0 + i < m) out[col0 + i] = (T)v[i];
                                }
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
        // 8. per-row outputs of the segment (mode 2: written by mode 1).  Mode
        //    1 also probes the visited set with each key as a keys-first probe
        //    does: claim an empty slot, or take an entry with the key's tag as
        //    the child's configuration, the earliest child of the chunk keeping
        //    an entry of the chunk (the row check settles it later).
        if (!ROWS && tid >= c && tid < cend) {
            const long long b = b0 + tid;
            const u64 key = fmix64(L.rowh[tid]) & a.hash_mask;
            a.hash[b] = key;
            a.cpar[b] = (int)p;
            a.ct[b] = my_t;
            if (KEYS && a.table) {
                const uint32_t tag = (uint32_t)(key >> 32);
                const u64 mine = ((u64)tag << 32) | (kStageBase + (uint32_t)b);
                u64 sl = key & a.slot_mask;
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
                        if (mine < e) atomicMin(&a.table[sl], mine);
                        placed = true;
                        break;
                    }
                    sl = (sl + 1) & a.slot_mask;
                }
                a.slot[b] = placed ? (uint32_t)sl : 0u;
                if (!placed) atomicOr((unsigned long long*)&a.ctr->probe_fail, 1ULL);
            }
        }
        // the last child of this segment, for the next reference child
        if constexpr (!KEYS) {
            for (int j = tid; j < m; j += blockDim.x) L.dp[j] = L.dgb[j];
            last_row = ROWS ? (const T*)L.rowdst[cend - 1] : stage + (b0 + cend - 1) * (long long)m;
            last_h = ROWS ? 0 : L.rowh[cend - 1];
        }
        last_p = p;
        last_u = ua + (u64)(len - 1);
        // next segment: the rest of this parent's canonical children, else the
        // next parent with one
        c = cend;
        ua += (u64)len;
        if (ua >= psi_p) {
            ++p;
            while (p < a.n && a.psi[p] == 0) ++p;
            ua = 0;
        }
        __syncthreads();
        if (c < rows && p >= a.n) break;  // unreachable while g0 + B <= sum of Psi
    }
    if (p >= a.n || past) break;
    }
    if (__syncthreads_or(ovf) && tid == 0) atomicOr((unsigned long long*)&a.ctr->overflow, 1ULL);
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
    const int tpb = a.tiles > 0 ? std::min(a.tiles, 64)
                                : (int)std::max<long long>(1, std::min<long long>(16, tiles / (4 * resident)));
    const unsigned blocks = (unsigned)((tiles + tpb - 1) / tpb);
#define SNP_I8(TT, NN, MM) hipLaunchKernelGGL((k_expand_int8<TT, NN, MM>), dim3(blocks), dim3(256), lds, st, s, a, tpb)
#define SNP_I8M(TT, NN)                   \
    do {                                  \
        if (a.mode == 1) SNP_I8(TT, NN, 1); \
        else if (a.mode == 2) SNP_I8(TT, NN, 2); \
        else SNP_I8(TT, NN, 0);           \
    } while (0)
    if (elem_bytes == 4) {
        if (wide) SNP_I8M(int32_t, 128);
        else SNP_I8M(int32_t, 64);
    } else {
        if (wide) SNP_I8M(uint16_t, 128);
        else SNP_I8M(uint16_t, 64);
    }
#undef SNP_I8M
#undef SNP_I8
    return hipGetLastError();
}

}  // namespace snp
