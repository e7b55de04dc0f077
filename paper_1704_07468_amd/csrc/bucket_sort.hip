// Per-bucket sort and segmentation of the partitioned g-mers (Section 2.2,
// step 3: for every reduced g-mer, the sequences that hold it and how often).
//
// A bucket holds the g-mers whose hashed reduced key shares its top B bits.
// Sorting it by the composite word (hash rest, then sequence id) puts equal
// reduced g-mers next to each other ("groups") and, inside a group, equal
// sequences next to each other ("runs").  The scan kernel files every
// non-empty bucket into a size class; then
//   * a bucket of at most 512 g-mers (256 with 64-bit composites) is sorted
//     by one wave, 64 * EL elements held in registers (EL per lane), by a
//     bitonic network whose exchanges are lane permutes (DPP row operations,
//     row / half-wave swaps) or register swaps;
//   * a bucket of at most 16384 g-mers (8192 with 64-bit composites) is
//     sorted the same way by 1, 2, .., 16 waves of a 1024-thread block, 1024
//     (512) elements a wave, the exchanges between waves going through LDS;
//   * a larger bucket is radix-sorted by a block in global memory.
// The sorted bucket goes to LDS and is segmented with ballot bitmaps of run
// and group starts: prefix popcounts give each run its entry index and each
// group its extent.
#include "common.h"
#include "launch.h"

namespace gk {

// ------------------------------------------------------------- classes --
// Composite words of at most 32 bits are sorted packed with the g-mer index
// as one 64-bit word (composite high); wider ones as (composite, index).
__device__ __forceinline__ int ceil_log2_u(uint32_t x) { return x <= 1 ? 0 : 32 - __clz(x - 1); }

__device__ __forceinline__ int bucket_class(uint32_t n, bool pk)
{
    if (n == 0) return -1;
    if (n <= (pk ? kSortWaveMaxPk : kSortWaveMaxWide)) {
        const int e = max(0, ceil_log2_u(n) - 6);  // log2 of elements per lane
        return pk ? e : 5 + e;                      // packed 0..4, wide 5..8
    }
    if (n <= (pk ? kSortBlockMaxPk : kSortBlockMaxWide)) {
        // log2 of waves per bucket (1024 packed / 512 wide elements a wave), 2..16
        const int e = ceil_log2_u(n) - (pk ? 11 : 10);  // 0..3
        return kSortClassWave + (pk ? e : 4 + e);
    }
    return kSortClassWave + kSortClassBlock + (pk ? 0 : 1);
}

// ---------------------------------------------------------- bucket scan --
// Exclusive scan of the bucket counts of one mask (one block per mask), and
// the filing of its non-empty buckets into the size-class lists.
__global__ __launch_bounds__(kThreads) void k_bucket_scan(const MaskWork *__restrict__ items, SortLists L)
{
    __shared__ uint32_t wsum[kWaves];
    __shared__ uint32_t ccnt[kSortClasses], cbase[kSortClasses];
    __shared__ uint32_t gsum[6];
    const int q = blockIdx.x;
    const MaskWork &W = items[q];
    const uint32_t nb = 1u << W.B;
    const uint32_t per = (nb + kThreads - 1) / kThreads;
    const uint32_t b0 = threadIdx.x * per;
    const gptr<uint32_t> bcnt = glb(W.bcnt), boff = glb(W.boff), bcur = glb(W.bcur);
    const gptr<uint32_t> lcnt = glb(L.cnt), list = glb(L.list);
    uint32_t loc = 0;
    for (uint32_t i = 0; i < per; ++i)
        if (b0 + i < nb) loc += bcnt[b0 + i];
    uint32_t tot;
    uint32_t run = block_excl_scan(loc, wsum, &tot);
    for (uint32_t i = 0; i < per; ++i)
        if (b0 + i < nb) {
            boff[b0 + i] = run;
            bcur[b0 + i] = run;
            run += bcnt[b0 + i];
        }
    if (threadIdx.x == 0) boff[nb] = tot;
    if (threadIdx.x < kSortClasses) ccnt[threadIdx.x] = 0;
    if (threadIdx.x < 6) gsum[threadIdx.x] = 0;
    __syncthreads();
    const bool pk = W.cb + W.ib <= 64;
    for (uint32_t b = threadIdx.x; b < nb; b += kThreads) {
        const uint32_t n = bcnt[b];
        const int c = bucket_class(n, pk);
        if (c >= 0) {
            atomicAdd(&ccnt[c], 1u);
            if (L.stat) {
                const int kind = c < kSortClassWave ? 0 : (c < kSortClassWave + kSortClassBlock ? 1 : 2);
                atomicAdd(&gsum[kind * 2 + (pk ? 0 : 1)], n);
            }
        } else if (W.gtab) {
            glb(W.bgrp)[b] = 0;
        }
    }
    __syncthreads();
    if (L.stat && threadIdx.x < 6 && gsum[threadIdx.x])
        g_atomic_add(glb(L.stat) + threadIdx.x, (unsigned long long)gsum[threadIdx.x]);
    if (threadIdx.x < kSortClasses) {
        const uint32_t c = ccnt[threadIdx.x];
        cbase[threadIdx.x] = c ? g_atomic_add(lcnt + threadIdx.x, c) : 0u;
        ccnt[threadIdx.x] = 0;
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < nb; b += kThreads) {
        const int c = bucket_class(bcnt[b], pk);
        if (c >= 0) {
            const uint32_t pos = cbase[c] + atomicAdd(&ccnt[c], 1u);
            if (pos < L.cap) list[(size_t)c * L.cap + pos] = ((uint32_t)q << kListBucketBits) | b;
        }
    }
}

// ------------------------------------------------------ bitonic network --
// The two values of the pair {i, i ^ J} that lane i belongs to (J < 64), all
// VALU: DPP quad permutes (J = 1, 2), DPP row rotations (J = 4: by 12 for the
// lanes with bit 2 clear, by 4 for the others; J = 8: by 8), and the gfx950
// row / half-wave swaps (J = 16, 32), which return the lower-index value
// first.  Order within the pair does not matter to the caller.
template <int J>
__device__ __forceinline__ void lane_pair(uint32_t x, uint32_t &a, uint32_t &b)
{
    if constexpr (J == 1) {
        a = x;
        b = (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false);  // quad_perm 1,0,3,2
    } else if constexpr (J == 2) {
        a = x;
        b = (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, false);  // quad_perm 2,3,0,1
    } else if constexpr (J == 4) {
        const uint32_t up = (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x12C, 0xF, 0xF, false);  // row_ror:12
        const uint32_t dn = (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x124, 0xF, 0xF, false);  // row_ror:4
        a = x;
        b = (__lane_id() & 4) ? dn : up;
    } else if constexpr (J == 8) {
        a = x;
        b = (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x128, 0xF, 0xF, false);  // row_ror:8
    } else if constexpr (J == 16) {
        const auto p = __builtin_amdgcn_permlane16_swap(x, x, false, false);
        a = p[0];
        b = p[1];
    } else {
        const auto p = __builtin_amdgcn_permlane32_swap(x, x, false, false);
        a = p[0];
        b = p[1];
    }
}

// Element order: packed words compare as integers; wide ones by composite,
// then g-mer index.  Real elements are pairwise distinct (distinct indices)
// and the padding (all ones: an index field of all ones, or index
// 0xFFFFFFFF, which no g-mer has) is strictly above them, so one comparison
// decides a pair.
template <bool PK>
__device__ __forceinline__ bool el_less(uint64_t ak, uint32_t av, uint64_t bk, uint32_t bv)
{
    if constexpr (PK) return ak < bk;
    else return (ak < bk) | ((ak == bk) & (av < bv));
}

// Exchange within the pair at distance J < 64.  keep_max: this lane keeps the
// larger element of its pair (the high end of an ascending pair or the low
// end of a descending one).
template <bool PK, int J>
__device__ __forceinline__ void exchange_lanes(uint64_t &key, uint32_t &val, bool keep_max)
{
    uint32_t ah, bh, al, bl;
    lane_pair<J>((uint32_t)(key >> 32), ah, bh);
    lane_pair<J>((uint32_t)key, al, bl);
    const uint64_t ak = ((uint64_t)ah << 32) | al, bk = ((uint64_t)bh << 32) | bl;
    uint32_t av = 0, bv = 0;
    if constexpr (!PK) lane_pair<J>(val, av, bv);
    const bool take_a = el_less<PK>(ak, av, bk, bv) != keep_max;
    key = take_a ? ak : bk;
    if constexpr (!PK) val = take_a ? av : bv;
}

// Elements are held blocked: lane l has elements i = ibase + EL l + e in its
// registers e = 0..EL-1, so the stages of distance below EL are register
// swaps and only the longer ones exchange between lanes.

// Stage of element distance J EL (lane distance J < 64) for every register.
// A pair is ascending when bit k of i is 0; k >= 2 J EL, so that bit belongs
// to ibase + EL l, the same for all registers of the lane.
template <bool PK, int EL, int J>
__device__ __forceinline__ void stage_lanes(uint64_t (&key)[EL], uint32_t (&val)[EL], uint32_t ibase, uint32_t k)
{
    const int lane = __lane_id();
    const bool upper = (lane & J) != 0;
    const bool asc = ((ibase + (uint32_t)(EL * lane)) & k) == 0;
    const bool keep_max = upper == asc;
#pragma unroll
    for (int e = 0; e < EL; ++e) exchange_lanes<PK, J>(key[e], val[e], keep_max);
}

// Stage of distance D < EL: registers e and e | D of the same lane.
template <bool PK, int EL, int D>
__device__ __forceinline__ void stage_regs(uint64_t (&key)[EL], uint32_t (&val)[EL], uint32_t ibase, uint32_t k)
{
    if constexpr (D < EL) {
        const uint32_t l0 = ibase + (uint32_t)(EL * __lane_id());
#pragma unroll
        for (int e = 0; e < EL; ++e) {
            if ((e & D) == 0) {
                const int e2 = e | D;
                const bool asc = ((l0 + (uint32_t)e) & k) == 0;
                const bool sw = el_less<PK>(key[e2], val[e2], key[e], val[e]) == asc;
                const uint64_t ka = key[e], kb = key[e2];
                key[e] = sw ? kb : ka;
                key[e2] = sw ? ka : kb;
                if constexpr (!PK) {
                    const uint32_t va = val[e], vb = val[e2];
                    val[e] = sw ? vb : va;
                    val[e2] = sw ? va : vb;
                }
            }
        }
    }
}

// Stage of distance j >= 64 EL: between waves of a block, through LDS.
template <bool PK, int EL>
__device__ __forceinline__ void stage_lds(uint64_t (&key)[EL], uint32_t (&val)[EL], uint64_t *kb, uint32_t *vb,
                                          uint32_t ibase, uint32_t k, uint32_t j)
{
    const uint32_t l0 = ibase + (uint32_t)(EL * __lane_id());
    __syncthreads();
#pragma unroll
    for (int e = 0; e < EL; ++e) {
        kb[l0 + e] = key[e];
        if constexpr (!PK) vb[l0 + e] = val[e];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < EL; ++e) {
        const uint32_t i = l0 + (uint32_t)e;
        const uint64_t yk = kb[i ^ j];
        uint32_t yv = 0;
        if constexpr (!PK) yv = vb[i ^ j];
        const bool keep_max = ((i & j) != 0) == ((i & k) == 0);
        const bool take = el_less<PK>(yk, yv, key[e], val[e]) != keep_max;
        key[e] = take ? yk : key[e];
        if constexpr (!PK) val[e] = take ? yv : val[e];
    }
}

// Bitonic sort of NW * 64 * EL elements, ascending in i; wave `wave` of the
// NW holds elements [wave * 64 EL, (wave + 1) * 64 EL).
template <bool PK, int EL, int NW>
__device__ __forceinline__ void bitonic_sort(uint64_t (&key)[EL], uint32_t (&val)[EL], uint64_t *kb, uint32_t *vb, int wave)
{
    constexpr uint32_t WSPAN = 64u * EL;
    constexpr uint32_t NP = WSPAN * NW;
    const uint32_t ibase = (uint32_t)wave * WSPAN;
    for (uint32_t k = 2; k <= NP; k <<= 1) {
        if constexpr (NW > 1)
            for (uint32_t j = k >> 1; j >= WSPAN; j >>= 1) stage_lds<PK, EL>(key, val, kb, vb, ibase, k, j);
        // lane stages, element distances WSPAN / 2 .. EL
        if (k > 32u * EL) stage_lanes<PK, EL, 32>(key, val, ibase, k);
        if (k > 16u * EL) stage_lanes<PK, EL, 16>(key, val, ibase, k);
        if (k > 8u * EL) stage_lanes<PK, EL, 8>(key, val, ibase, k);
        if (k > 4u * EL) stage_lanes<PK, EL, 4>(key, val, ibase, k);
        if (k > 2u * EL) stage_lanes<PK, EL, 2>(key, val, ibase, k);
        if (k > 1u * EL) stage_lanes<PK, EL, 1>(key, val, ibase, k);
        // register stages, distances EL / 2 .. 1
        if (k > 8) stage_regs<PK, EL, 8>(key, val, ibase, k);
        if (k > 4) stage_regs<PK, EL, 4>(key, val, ibase, k);
        if (k > 2) stage_regs<PK, EL, 2>(key, val, ibase, k);
        stage_regs<PK, EL, 1>(key, val, ibase, k);
    }
}

// ----------------------------------------------------------- segmentation --
// One 64-bit word per 64 sorted positions: run starts (rbm), group starts
// (gbm), positions whose composite recurs 127 positions later, i.e. that lie
// in a run of more than 127 g-mers (lbm), and starts of candidate groups for
// the count matrix (cbm), with their exclusive prefix popcounts, the position
// of the next run / group start at or after each word and of the last group
// start before it (n, resp. none, when there is none); slot: one word per
// candidate group.
template <int NWORDS, int NSLOT>
struct SegLds {
    uint64_t rbm[NWORDS], gbm[NWORDS], lbm[NWORDS], cbm[NWORDS];
    uint32_t rpre[NWORDS + 1], gpre[NWORDS + 1], cpre[NWORDS + 1];
    uint32_t nextr[NWORDS + 1], nextg[NWORDS + 1], prevg[NWORDS + 1];
    uint32_t inner;  // some full word holds no group start (lies inside one group)
    uint32_t slot[NSLOT];
};

template <int NW>
__device__ __forceinline__ void seg_sync()
{
    if constexpr (NW > 1) __syncthreads();
    else wave_sync();
}

// Wave-wide inclusive prefix max and suffix max of unsigned values (0 is the
// identity): DPP shifts within rows of 16 lanes, then the row totals.
__device__ __forceinline__ uint32_t wave_prefix_max_u(uint32_t x)
{
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false));  // row_shr:1
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false));  // row_shr:2
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false));  // row_shr:4
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false));  // row_shr:8
    const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)x, 15);
    const uint32_t r1 = max(r0, (uint32_t)__builtin_amdgcn_readlane((int)x, 31));
    const uint32_t r2 = max(r1, (uint32_t)__builtin_amdgcn_readlane((int)x, 47));
    const int row = __lane_id() >> 4;
    return max(x, row == 0 ? 0u : row == 1 ? r0 : row == 2 ? r1 : r2);
}
__device__ __forceinline__ uint32_t wave_suffix_max_u(uint32_t x)
{
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x101, 0xF, 0xF, false));  // row_shl:1
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x102, 0xF, 0xF, false));  // row_shl:2
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x104, 0xF, 0xF, false));  // row_shl:4
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x108, 0xF, 0xF, false));  // row_shl:8
    const uint32_t r3 = (uint32_t)__builtin_amdgcn_readlane((int)x, 48);
    const uint32_t r2 = max(r3, (uint32_t)__builtin_amdgcn_readlane((int)x, 32));
    const uint32_t r1 = max(r2, (uint32_t)__builtin_amdgcn_readlane((int)x, 16));
    const int row = __lane_id() >> 4;
    return max(x, row == 3 ? 0u : row == 2 ? r3 : row == 1 ? r2 : r1);
}
__device__ __forceinline__ uint32_t wave_suffix_min(uint32_t x) { return ~wave_suffix_max_u(~x); }
__device__ __forceinline__ int wave_prefix_max(int x)  // x >= -1
{
    return (int)wave_prefix_max_u((uint32_t)(x + 1)) - 1;
}
// The value of lane + 1 (lane 63: 0) and of lane - 1 (lane 0: 0).
__device__ __forceinline__ uint32_t from_next_lane(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x130, 0xF, 0xF, false);  // wave_shl:1
}
__device__ __forceinline__ uint32_t from_prev_lane(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x138, 0xF, 0xF, false);  // wave_shr:1
}

__device__ __forceinline__ uint32_t first_bit(int w, uint64_t m) { return (uint32_t)(w * 64 + __ffsll((long long)m) - 1); }
__device__ __forceinline__ int last_bit(int w, uint64_t m) { return w * 64 + 63 - (int)__clzll((long long)m); }

// One wave: prefix popcounts of rbm and gbm, next run / group starts and the
// last group start before each word, over nwords words.
template <int NWORDS, int NSLOT>
__device__ __forceinline__ void scan_words(SegLds<NWORDS, NSLOT> &S, int nwords, uint32_t n)
{
    constexpr int PER = (NWORDS + 63) / 64;
    const int lane = __lane_id();
    uint32_t rc = 0, gc = 0, fr = n, fg = n;
    int lg = -1;
    bool inner = false;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int w = lane * PER + p;
        if (w < nwords && S.gbm[w]) lg = last_bit(w, S.gbm[w]);
        if (w < nwords && (uint32_t)(w + 1) * 64u <= n && !S.gbm[w]) inner = true;
    }
    const bool any_inner = __ballot(inner) != 0;
#pragma unroll
    for (int p = PER - 1; p >= 0; --p) {
        const int w = lane * PER + p;
        if (w < nwords) {
            const uint64_t r = S.rbm[w], g = S.gbm[w];
            rc += __popcll(r);
            gc += __popcll(g);
            if (r) fr = first_bit(w, r);
            if (g) fg = first_bit(w, g);
        }
    }
    const uint32_t ri = wave_incl_scan(rc), gi = wave_incl_scan(gc);
    uint32_t rx = ri - rc, gx = gi - gc;
    const uint32_t sr = wave_suffix_min(fr), sg = wave_suffix_min(fg);
    uint32_t ar = from_next_lane(sr), ag = from_next_lane(sg);
    if (lane == 63) ar = ag = n;
    int pg = (int)from_prev_lane((uint32_t)wave_prefix_max(lg));
    if (lane == 0) pg = -1;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int w = lane * PER + p;
        if (w < nwords) {
            S.rpre[w] = rx;
            S.gpre[w] = gx;
            S.prevg[w] = (uint32_t)pg;
            rx += __popcll(S.rbm[w]);
            gx += __popcll(S.gbm[w]);
            if (S.gbm[w]) pg = last_bit(w, S.gbm[w]);
        }
    }
#pragma unroll
    for (int p = PER - 1; p >= 0; --p) {
        const int w = lane * PER + p;
        if (w < nwords) {
            const uint64_t r = S.rbm[w], g = S.gbm[w];
            if (r) ar = first_bit(w, r);
            if (g) ag = first_bit(w, g);
            S.nextr[w] = ar;
            S.nextg[w] = ag;
        }
    }
    const uint32_t R = (uint32_t)__builtin_amdgcn_readlane((int)ri, 63), G = (uint32_t)__builtin_amdgcn_readlane((int)gi, 63);
    if (lane == 0) {
        S.rpre[nwords] = R;
        S.gpre[nwords] = G;
        S.nextr[nwords] = n;
        S.nextg[nwords] = n;
        S.inner = any_inner ? 1u : 0u;
    }
}

// One wave: exclusive prefix popcounts of cbm, the total at cpre[nwords].
template <int NWORDS, int NSLOT>
__device__ __forceinline__ void scan_cand(SegLds<NWORDS, NSLOT> &S, int nwords)
{
    constexpr int PER = (NWORDS + 63) / 64;
    const int lane = __lane_id();
    uint32_t cc = 0;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int w = lane * PER + p;
        if (w < nwords) cc += __popcll(S.cbm[w]);
    }
    const uint32_t ci = wave_incl_scan(cc);
    uint32_t cx = ci - cc;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int w = lane * PER + p;
        if (w < nwords) {
            S.cpre[w] = cx;
            cx += __popcll(S.cbm[w]);
        }
    }
    const uint32_t C = (uint32_t)__builtin_amdgcn_readlane((int)ci, 63);
    if (lane == 0) S.cpre[nwords] = C;
}

struct RunAt {
    uint32_t r;    // run index in the bucket
    uint32_t cnt;  // g-mers in the run
    uint32_t len;  // runs from this one to the group end
    uint32_t gi;   // group index in the bucket
    uint32_t gs;   // position of the group's first g-mer
    uint32_t gend; // position after the group's last g-mer
};

// The run starting at sorted position i (word w = i / 64, bit b = i % 64).
template <int NWORDS, int NSLOT>
__device__ __forceinline__ RunAt run_at(const SegLds<NWORDS, NSLOT> &S, int w, int b, uint32_t i, uint32_t n, uint32_t R)
{
    const uint64_t rb = S.rbm[w], gb = S.gbm[w];
    const uint64_t le = (b == 63) ? ~0ull : ((2ull << b) - 1ull);
    const uint64_t gt = ~le;
    RunAt a;
    a.r = S.rpre[w] + (uint32_t)__popcll(rb & (le >> 1));
    const uint64_t mr = rb & gt, mg = gb & gt, ml = gb & le;
    const uint32_t end = mr ? first_bit(w, mr) : S.nextr[w + 1];
    const uint32_t gend = mg ? first_bit(w, mg) : S.nextg[w + 1];
    a.cnt = end - i;
    uint32_t rend = R;
    if (gend < n) {
        const int gw = (int)(gend >> 6);
        rend = S.rpre[gw] + (uint32_t)__popcll(S.rbm[gw] & ((1ull << (gend & 63)) - 1ull));
    }
    a.len = rend - a.r;
    a.gi = S.gpre[w] + (uint32_t)__popcll(ml) - 1u;
    a.gs = ml ? (uint32_t)last_bit(w, ml) : S.prevg[w];
    a.gend = gend;
    return a;
}

__device__ __forceinline__ bool bit_at(const uint64_t *bm, uint32_t i) { return (bm[i >> 6] >> (i & 63)) & 1ull; }

// The tables of word w, read once by the wave (w is wave-uniform) and kept
// in scalar registers.
struct WordAt {
    uint64_t rb, gb;
    uint32_t rpre, gpre, nextr1, nextg1, prevg;
};

__device__ __forceinline__ uint64_t uniform64(uint64_t x)
{
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32)) << 32) |
           (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
}
__device__ __forceinline__ uint32_t uniform32(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }

template <int NWORDS, int NSLOT>
__device__ __forceinline__ WordAt word_at(const SegLds<NWORDS, NSLOT> &S, int w)
{
    WordAt u;
    u.rb = uniform64(S.rbm[w]);
    u.gb = uniform64(S.gbm[w]);
    u.rpre = uniform32(S.rpre[w]);
    u.gpre = uniform32(S.gpre[w]);
    u.nextr1 = uniform32(S.nextr[w + 1]);
    u.nextg1 = uniform32(S.nextg[w + 1]);
    u.prevg = uniform32(S.prevg[w]);
    return u;
}

// run_at with the word's tables already at hand.
template <int NWORDS, int NSLOT>
__device__ __forceinline__ RunAt run_at_w(const SegLds<NWORDS, NSLOT> &S, const WordAt &u, int w, int b, uint32_t i,
                                          uint32_t n, uint32_t R)
{
    const uint64_t le = (b == 63) ? ~0ull : ((2ull << b) - 1ull);
    const uint64_t gt = ~le;
    RunAt a;
    a.r = u.rpre + (uint32_t)__popcll(u.rb & (le >> 1));
    const uint64_t mr = u.rb & gt, mg = u.gb & gt, ml = u.gb & le;
    const uint32_t end = mr ? first_bit(w, mr) : u.nextr1;
    const uint32_t gend = mg ? first_bit(w, mg) : u.nextg1;
    a.cnt = end - i;
    uint32_t rend = R;
    if (gend < n) {
        const int gw = (int)(gend >> 6);
        rend = S.rpre[gw] + (uint32_t)__popcll(S.rbm[gw] & ((1ull << (gend & 63)) - 1ull));
    }
    a.len = rend - a.r;
    a.gi = u.gpre + (uint32_t)__popcll(ml) - 1u;
    a.gs = ml ? (uint32_t)last_bit(w, ml) : u.prevg;
    a.gend = gend;
    return a;
}

// Candidate slot of the group starting at position gs (a set bit of cbm).
template <int NWORDS, int NSLOT>
__device__ __forceinline__ uint32_t cand_slot(const SegLds<NWORDS, NSLOT> &S, uint32_t gs)
{
    const int cw = (int)(gs >> 6);
    return S.cpre[cw] + (uint32_t)__popcll(S.cbm[cw] & ((1ull << (gs & 63)) - 1ull));
}

// Adds each lane's diagonal term v (0: none) to counter q.  The terms of a
// wave often belong to few sequences (a query batch: every run has one of
// few sequence ids), so that lane-by-lane atomics would contend on few
// addresses: the wave sums the terms of one sequence at a time and adds each
// sum once, for up to 16 sequences and while a sequence has more than one
// term; the remaining terms go lane by lane.
__device__ __forceinline__ void diag_add(gptr<uint32_t> diag, uint32_t nseq, uint32_t v, uint32_t q, uint32_t *dl,
                                         uint32_t dofs)
{
    if (dl) {  // the block's LDS sums (few counters in all)
        if (v != 0 && q < nseq) atomicAdd(&dl[dofs + q], v);
        return;
    }
    uint64_t act = __ballot(v != 0);
#pragma unroll 1
    for (int k = 0; k < 16 && act; ++k) {
        const uint32_t q0 = (uint32_t)__builtin_amdgcn_readlane((int)q, __ffsll((long long)act) - 1);
        const bool mine = v != 0 && q == q0;
        const uint64_t mm = __ballot(mine);
        const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(mine ? v : 0u), 63);
        if (__lane_id() == 0 && q0 < nseq) g_atomic_add(diag + q0, tot);
        if (mine) v = 0;
        act = __ballot(v != 0);
        if (__popcll(mm) == 1) break;  // sequences mostly distinct: the rest lane by lane
    }
    if (v != 0 && q < nseq) g_atomic_add(diag + q, v);
}

// Runs and groups of one sorted bucket in LDS (kb: packed words or
// composites, vb: indices of wide ones), segmented by the NW waves of its
// group (wave = the wave's index in the group).  Writes one run entry
// (sequence | count << sb) per run at E[base + run], so each group's entries
// are contiguous and sequence-sorted; per g-mer its info -- for the first
// g-mer of a run (entry index, runs to the group end | count << (sb+1)), for
// the others (0, 0); with W.inl a run two entries from its group end carries
// that last entry (sequence | count << sb) instead of its index.  Groups with
// at least tau runs and every count <= 127 become rows of the int8 count
// matrix instead (info length 0), as far as NSLOT candidate groups per bucket
// (otherwise all of the bucket's groups stay on the exact sparse path).  With
// gtab, lists the groups (hash rest, first entry, end entry); with diag, adds
// count^2 per run to its sequence's diagonal counter.  n = 0 does nothing but
// takes part in the barriers: every barrier is reached by every wave of the
// block, whatever its bucket.
// LP > 0: the sorted elements are keys composite << LP | position in the
// bucket, the g-mer indices in vb by position.
template <bool PK, int NW, int NWORDS, int NSLOT, int LP = 0>
__device__ __forceinline__ void segment(const MaskWork &W, uint32_t bucket, uint32_t base, uint32_t n, const uint64_t *kb,
                                        const uint32_t *vb, SegLds<NWORDS, NSLOT> &S, int wave, uint32_t *dl,
                                        const uint32_t *diag0)
{
    constexpr int NT = NW * 64;
    const int lane = __lane_id();
    const int tid = wave * 64 + lane;
    // the mask's fields, read once: stores through its pointers could
    // otherwise alias the descriptor and force reloads after every store
    const int sb = W.sb;
    const gptr<uint32_t> E = glb(W.E);
    const gptr<uint16_t> E16 = glb((uint16_t *)W.E);
    const gptr<uint2> info = glb(W.info);
    const gptr<int8_t> D = glb(W.D);
    const gptr<uint32_t> dcount = glb(W.dcount);
    const gptr<uint32_t> diag = glb(W.diag);
    const gptr<uint4> gtab = glb(W.gtab);
    const gptr<uint32_t> bgrp = glb(W.bgrp);
    const uint32_t T = W.T, Nseq = (uint32_t)W.N, dcap = W.dcap, dstride = W.dstride;
    const int tau = W.tau, inl = W.inl, i4 = W.i4;
    const gptr<uint32_t> info4 = (gptr<uint32_t>)info, lenx = info4 + T;
    const uint64_t sidmask = bits_mask(sb);
    const int ib = W.ib;
    const uint64_t ibmask = bits_mask(ib);
    const int nwords = (int)((n + 63) >> 6);
    auto comp_at = [&](uint32_t i) -> uint64_t {
        if constexpr (LP > 0) return kb[i] >> LP;
        else return PK ? (kb[i] >> ib) : kb[i];
    };
#pragma unroll 1
    for (int w = wave; w < nwords; w += NW) {
        const uint32_t i = (uint32_t)w * 64u + (uint32_t)lane;
        bool rs = false, gs = false, lr = false;
        if (i < n) {
            const uint64_t c = comp_at(i);
            if (i == 0) {
                rs = gs = true;
            } else {
                const uint64_t p = comp_at(i - 1);
                rs = c != p;
                gs = (c >> sb) != (p >> sb);
            }
            lr = i + 127u < n && comp_at(i + 127u) == c;
        }
        const uint64_t rb = __ballot(rs), gb = __ballot(gs), lb = __ballot(lr);
        if (lane == 0) {
            S.rbm[w] = rb;
            S.gbm[w] = gb;
            S.lbm[w] = lb;
        }
    }
    seg_sync<NW>();
    if (wave == 0) scan_words<NWORDS, NSLOT>(S, nwords, n);
    seg_sync<NW>();
    const uint32_t R = S.rpre[nwords], G = S.gpre[nwords];
    // count-matrix candidates: groups with at least tau runs, none of them
    // longer than 127 g-mers.  Such a group spans at least tau positions;
    // from 127 on, that covers one full word without a group start, so
    // buckets without such a word are skipped.
    const bool dense_on = n > 0 && tau > 0 && D != nullptr && R >= (uint32_t)tau && (tau < 127 || S.inner);
    if (dense_on) {
#pragma unroll 1
        for (int w = wave; w < nwords; w += NW) {
            const uint32_t i = (uint32_t)w * 64u + (uint32_t)lane;
            const WordAt u = word_at(S, w);
            bool c = false;
            if (i < n && ((u.gb >> lane) & 1ull)) {
                const uint64_t gt = lane == 63 ? 0ull : (~0ull << (lane + 1));
                const uint64_t mg = u.gb & gt;
                const uint32_t gend = mg ? first_bit(w, mg) : u.nextg1;
                if (gend - i >= (uint32_t)tau) {  // long enough in positions: count its runs
                    const uint32_t r0 = u.rpre + (uint32_t)__popcll(u.rb & ~(gt | (1ull << lane)));
                    uint32_t r1 = R;
                    if (gend < n) {
                        const int gw = (int)(gend >> 6);
                        r1 = S.rpre[gw] + (uint32_t)__popcll(S.rbm[gw] & ((1ull << (gend & 63)) - 1ull));
                    }
                    if (r1 - r0 >= (uint32_t)tau) {
                        // no position of the group in a run longer than 127
                        bool ok = true;
                        for (int x = w; x <= (int)((gend - 1) >> 6) && ok; ++x) {
                            uint64_t m = S.lbm[x];
                            if (x == w) m &= ~0ull << lane;
                            if (x == (int)((gend - 1) >> 6) && (gend & 63)) m &= (1ull << (gend & 63)) - 1ull;
                            ok = m == 0;
                        }
                        c = ok;
                    }
                }
            }
            const uint64_t cb = __ballot(c);
            if (lane == 0) S.cbm[w] = cb;
        }
    }
    seg_sync<NW>();
    if (dense_on && wave == 0) scan_cand<NWORDS, NSLOT>(S, nwords);
    seg_sync<NW>();
    const uint32_t ncand = dense_on ? S.cpre[nwords] : 0u;
    const bool dense = ncand > 0 && ncand <= (uint32_t)NSLOT;
    if (dense) {  // every candidate takes a count-matrix row while rows last
        for (uint32_t s = (uint32_t)tid; s < ncand; s += NT) {
            uint32_t row = g_atomic_add(dcount, 1u);
            if (row >= dcap) row = 0xFFFFFFFFu;
            S.slot[s] = row;
        }
    }
    seg_sync<NW>();
#pragma unroll 2
    for (int w = wave; w < nwords; w += NW) {
        const uint32_t i = (uint32_t)w * 64u + (uint32_t)lane;
        const WordAt u = word_at(S, w);
        uint32_t dv = 0, dq = 0;  // this lane's diagonal term count^2 and its sequence
        if (i < n) {
            uint32_t idx;
            if constexpr (LP > 0) idx = vb[(uint32_t)kb[i] & ((1u << LP) - 1u)];
            else idx = PK ? (uint32_t)(kb[i] & ibmask) : vb[i];
            if (!((u.rb >> lane) & 1ull)) {
                if (idx < T && !i4) st_u2(info, idx, 0u, 0u);  // (4-byte records start zeroed)
            } else {
                const RunAt a = run_at_w<NWORDS, NSLOT>(S, u, w, lane, i, n, R);
                const uint64_t c = comp_at(i);
                const uint32_t sid = (uint32_t)(c & sidmask);
                const uint32_t ei = base + a.r;
                if (i4) store_entry16(E16, T, ei, sid, a.cnt, sb);
                else E[ei] = sid | (a.cnt << sb);
                uint32_t y = a.len | (a.cnt << (sb + 1));
                if (dense && a.gs < n && bit_at(S.cbm, a.gs)) {
                    const uint32_t row = S.slot[cand_slot(S, a.gs)];
                    if (row != 0xFFFFFFFFu) {
                        if (sid < Nseq && row < dcap) D[tiled_offset(sid, row, dstride)] = (int8_t)a.cnt;
                        y = 0;
                    }
                }
                uint32_t x = ei;
                if (inl && y != 0 && a.len == 2) {  // the group's last run, inline
                    const uint32_t nx = i + a.cnt;
                    x = (uint32_t)(comp_at(nx) & sidmask) | ((a.gend - nx) << sb);
                }
                if (idx < T) {
                    if (i4) {
                        const uint32_t rec = pack_info4(y ? a.len : 0u, a.cnt, ei, inl && a.len == 2, x, sb, lenx);
                        if (rec) info4[idx] = rec;
                    } else {
                        st_u2(info, idx, x, y);
                    }
                }
                dv = a.cnt * a.cnt;
                dq = sid;
                if (gtab && a.gs == i) {
                    const uint64_t hr = c >> sb;
                    st_u4(gtab, base + a.gi, (uint32_t)hr, (uint32_t)(hr >> 32), ei, ei + a.len);
                }
            }
        }
        if (diag) diag_add(diag, Nseq, dv, dq, dl, (uint32_t)(W.diag - diag0));
    }
    if (gtab && n > 0 && tid == 0) bgrp[bucket] = G;
}

// Load a bucket's (composite, index) pairs into registers, padding with the
// largest element.  The loads are coalesced (register e of lane l takes
// element ibase + 64 e + l); which slot holds which element does not matter
// before the sort.
template <bool PK, int EL>
__device__ __forceinline__ void load_bucket(const MaskWork &W, uint32_t base, uint32_t n, uint32_t ibase, uint64_t (&key)[EL],
                                            uint32_t (&val)[EL])
{
    const int lane = __lane_id();
    const gptr<const uint64_t> comp = glb((const uint64_t *)W.comp);
    const gptr<const uint32_t> gidx = glb((const uint32_t *)W.idx);
#pragma unroll
    for (int e = 0; e < EL; ++e) {
        const uint32_t i = ibase + (uint32_t)(e * 64 + lane);
        key[e] = ~0ull;
        val[e] = 0xFFFFFFFFu;
        if (i < n) {
            key[e] = comp[base + i];  // packed: composite << 32 | index
            if constexpr (!PK) val[e] = gidx[base + i];
        }
    }
}

// Store the sorted elements held in registers (blocked: i = ibase + EL lane
// + e) to LDS.
template <bool PK, int EL>
__device__ __forceinline__ void store_sorted(const uint64_t (&key)[EL], const uint32_t (&val)[EL], uint32_t ibase, uint32_t n,
                                             uint64_t *kb, uint32_t *vb)
{
    const int lane = __lane_id();
#pragma unroll
    for (int e = 0; e < EL; ++e) {
        const uint32_t i = ibase + (uint32_t)(EL * lane + e);
        if (i < n) {
            kb[i] = key[e];
            if constexpr (!PK) vb[i] = val[e];
        }
    }
}

// ------------------------------------------------------ wave kernel --
// Two instances: the small one takes packed buckets of up to 512 g-mers and
// wide ones of up to 256, the big one packed 1024 and wide 512 (8 KB of
// elements per wave, fewer waves per CU).
constexpr int kWaveSlots = 128;

template <bool BIG>
struct WaveLds {
    static constexpr int KB = BIG ? 1024 : 512;      // packed elements
    static constexpr int WIDE = BIG ? 512 : 256;     // wide elements (then their indices)
    uint64_t kb[KB];
    SegLds<KB / 64, kWaveSlots> S;
};

template <bool BIG, bool PK, int EL>
__device__ __forceinline__ void wave_bucket(const MaskWork &W, uint32_t bucket, WaveLds<BIG> &lds, uint32_t *dl,
                                            const uint32_t *diag0)
{
    const gptr<const uint32_t> boff = glb((const uint32_t *)W.boff);
    const uint32_t base = boff[bucket];
    const uint32_t n = boff[bucket + 1] - base;
    if (n == 0 || n > 64u * EL) return;
    uint32_t *vb = reinterpret_cast<uint32_t *>(lds.kb + WaveLds<BIG>::WIDE);
    if constexpr (!PK) {
        // wide composites short enough to share 63 bits with the position in
        // the bucket: sort those keys on the packed network (one compare, no
        // index to carry), the g-mer indices wait in LDS by position
        constexpr int LP = 6 + (EL >= 8 ? 3 : EL >= 4 ? 2 : EL >= 2 ? 1 : 0);
        if (W.cb + LP <= 63) {
            const gptr<const uint64_t> comp = glb((const uint64_t *)W.comp);
            const gptr<const uint32_t> gidx = glb((const uint32_t *)W.idx);
            const int lane = __lane_id();
            uint64_t key[EL];
            uint32_t val[EL];
#pragma unroll
            for (int e = 0; e < EL; ++e) {
                const uint32_t i = (uint32_t)(e * 64 + lane);
                key[e] = ~0ull;  // padding, above every real key
                val[e] = 0;
                if (i < n) {
                    key[e] = (comp[base + i] << LP) | i;
                    vb[i] = gidx[base + i];
                }
            }
            bitonic_sort<true, EL, 1>(key, val, nullptr, nullptr, 0);
            store_sorted<true, EL>(key, val, 0, n, lds.kb, vb);
            wave_sync();
            segment<false, 1, WaveLds<BIG>::KB / 64, kWaveSlots, LP>(W, bucket, base, n, lds.kb, vb, lds.S, 0, dl, diag0);
            wave_sync();
            return;
        }
    }
    {
        uint64_t key[EL];
        uint32_t val[EL];
        load_bucket<PK, EL>(W, base, n, 0, key, val);
        bitonic_sort<PK, EL, 1>(key, val, nullptr, nullptr, 0);
        store_sorted<PK, EL>(key, val, 0, n, lds.kb, vb);
    }
    wave_sync();
    segment<PK, 1, WaveLds<BIG>::KB / 64, kWaveSlots>(W, bucket, base, n, lds.kb, vb, lds.S, 0, dl, diag0);
    wave_sync();
}

// Zero / flush the block's LDS diagonal sums (L.ndiag words of dynamic LDS).
template <int NT>
__device__ __forceinline__ uint32_t *diag_lds_begin(const SortLists &L, uint32_t *dyn)
{
    if (!L.ndiag) return nullptr;
    for (uint32_t i = threadIdx.x; i < L.ndiag; i += NT) dyn[i] = 0;
    __syncthreads();
    return dyn;
}
template <int NT>
__device__ __forceinline__ void diag_lds_end(const SortLists &L, const uint32_t *dl)
{
    if (!dl) return;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < L.ndiag; i += NT)
        if (dl[i]) g_atomic_add(glb(L.diag0) + i, dl[i]);
}

// Each wave takes the buckets of its instance's classes in a fixed stride
// over their concatenation, largest class first.
template <bool BIG>
__global__ __launch_bounds__(kThreads) void k_sort_wave(const MaskWork *__restrict__ items, SortLists L)
{
    __shared__ WaveLds<BIG> lds[kWaves];
    extern __shared__ uint32_t dyn_lds[];
    uint32_t *dl = diag_lds_begin<kThreads>(L, dyn_lds);
    // class ids: packed 64..1024 are 0..4, wide 64..512 are 5..8
    constexpr int NC = BIG ? 2 : 7;
    constexpr int order_small[7] = {3, 7, 2, 6, 1, 5, 0};  // packed 512, wide 256, packed 256, ...
    constexpr int order_big[2] = {4, 8};                   // packed 1024, wide 512
    const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // wave-uniform
    const uint32_t gw = blockIdx.x * kWaves + wid, nw = gridDim.x * kWaves;
    uint32_t cum[NC + 1];
    cum[0] = 0;
    const gptr<const uint32_t> lcnt = glb((const uint32_t *)L.cnt), list = glb((const uint32_t *)L.list);
#pragma unroll
    for (int s = 0; s < NC; ++s) cum[s + 1] = cum[s] + min(lcnt[BIG ? order_big[s] : order_small[s]], L.cap);
    for (uint32_t t = gw; t < cum[NC]; t += nw) {
        int s = 0;
#pragma unroll
        for (int q = 1; q < NC; ++q) s += (t >= cum[q]) ? 1 : 0;
        uint32_t off = 0;
        int c = 0;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            off = (q == s) ? cum[q] : off;
            c = (q == s) ? (BIG ? order_big[q] : order_small[q]) : c;
        }
        const uint32_t ent = list[(size_t)c * L.cap + (t - off)];
        const MaskWork &W = items[ent >> kListBucketBits];
        const uint32_t bucket = ent & kListBucketMask;
        if (bucket >= (1u << W.B)) continue;
        if constexpr (BIG) {
            if (c == 4) wave_bucket<true, true, 16>(W, bucket, lds[wid], dl, L.diag0);
            else wave_bucket<true, false, 8>(W, bucket, lds[wid], dl, L.diag0);
        } else {
            switch (c) {
            case 0: wave_bucket<false, true, 1>(W, bucket, lds[wid], dl, L.diag0); break;
            case 1: wave_bucket<false, true, 2>(W, bucket, lds[wid], dl, L.diag0); break;
            case 2: wave_bucket<false, true, 4>(W, bucket, lds[wid], dl, L.diag0); break;
            case 3: wave_bucket<false, true, 8>(W, bucket, lds[wid], dl, L.diag0); break;
            case 5: wave_bucket<false, false, 1>(W, bucket, lds[wid], dl, L.diag0); break;
            case 6: wave_bucket<false, false, 2>(W, bucket, lds[wid], dl, L.diag0); break;
            default: wave_bucket<false, false, 4>(W, bucket, lds[wid], dl, L.diag0); break;
            }
        }
    }
    diag_lds_end<kThreads>(L, dl);
}

// ------------------------------------------------------ block kernel --
// A 1024-thread block sorts G = 16 / NW buckets of one class side by side:
// each group of NW waves holds one bucket, 64 * EL elements per wave (EL = 16
// packed, 8 wide), so only the merges beyond one wave's share go through LDS.
// All groups run the same network and reach the same barriers.
constexpr int kSortBlockThreads = 1024;
constexpr int kSortBlockWaves = kSortBlockThreads / 64;
constexpr int kBlockSlots = 1024;  // count-matrix candidate slots per block

template <int NWORDS, int NSLOT>
constexpr size_t seg_bytes() { return sizeof(SegLds<NWORDS, NSLOT>); }

struct BlockLds {
    uint64_t buf[kSortBlockMaxPk];  // exchange buffers, then the sorted buckets
    // per-group segmentation scratch (largest: 8 groups of 32 words)
    uint64_t seg[(8 * seg_bytes<32, kBlockSlots / 8>() + 7) / 8];
};

template <bool PK, int NW>
__device__ __forceinline__ void block_buckets(const MaskWork *__restrict__ items, gptr<const uint32_t> ents, int nb, BlockLds &lds,
                                              uint32_t *dl, const uint32_t *diag0)
{
    constexpr int EL = PK ? 16 : 8;
    constexpr int NP = NW * 64 * EL;
    constexpr int G = kSortBlockWaves / NW;
    constexpr int NWORDS = NP / 64;
    constexpr int NSLOT = kBlockSlots / G;
    using Seg = SegLds<NWORDS, NSLOT>;
    static_assert(sizeof(Seg) * G <= sizeof(lds.seg), "segmentation scratch");
    static_assert((PK ? 8 : 12) * NP * G <= (int)sizeof(lds.buf), "exchange buffers");
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int gi = wave / NW, wg = wave % NW;
    // this group's bucket (none: n = 0, the first bucket's mask stands in)
    const uint32_t ent = ents[gi < nb ? gi : 0];
    const MaskWork &W = items[ent >> kListBucketBits];
    const uint32_t bucket = ent & kListBucketMask;
    uint32_t base = 0, n = 0;
    if (gi < nb && bucket < (1u << W.B)) {
        const gptr<const uint32_t> boff = glb((const uint32_t *)W.boff);
        base = boff[bucket];
        n = min(boff[bucket + 1] - base, (uint32_t)NP);
    }
    uint64_t *kb = lds.buf + (size_t)gi * NP;
    uint32_t *vb = reinterpret_cast<uint32_t *>(lds.buf + (size_t)G * NP) + (size_t)gi * NP;  // wide only
    Seg &S = *reinterpret_cast<Seg *>(reinterpret_cast<char *>(lds.seg) + (size_t)gi * sizeof(Seg));
    {
        uint64_t key[EL];
        uint32_t val[EL];
        const uint32_t ibase = (uint32_t)wg * 64u * EL;
        load_bucket<PK, EL>(W, base, n, ibase, key, val);
        bitonic_sort<PK, EL, NW>(key, val, kb, vb, wg);
        __syncthreads();  // the last exchange reads are done
        store_sorted<PK, EL>(key, val, ibase, n, kb, vb);
    }
    __syncthreads();
    segment<PK, NW, NWORDS, NSLOT>(W, bucket, base, n, kb, vb, S, wg, dl, diag0);
}

// Blocks take groups of buckets of one block class from a shared ticket
// counter, largest class first.
__global__ __launch_bounds__(kSortBlockThreads) void k_sort_block(const MaskWork *__restrict__ items, SortLists L)
{
    __shared__ BlockLds lds;
    __shared__ uint32_t ticket;
    extern __shared__ uint32_t dyn_lds[];
    uint32_t *dl = diag_lds_begin<kSortBlockThreads>(L, dyn_lds);
    // class offsets within the block classes, largest first: packed 16384,
    // wide 8192, packed 8192, wide 4096, ..., packed 2048, wide 1024; buckets
    // per block = 16 / waves per bucket
    constexpr int order[kSortClassBlock] = {3, 7, 2, 6, 1, 5, 0, 4};
    constexpr int gsz[kSortClassBlock] = {1, 1, 2, 2, 4, 4, 8, 8};
    uint32_t cum[kSortClassBlock + 1];
    cum[0] = 0;
    const gptr<uint32_t> lcnt = glb(L.cnt);
#pragma unroll
    for (int s = 0; s < kSortClassBlock; ++s)
        cum[s + 1] = cum[s] + (min(lcnt[kSortClassWave + order[s]], L.cap) + gsz[s] - 1) / gsz[s];
    const uint32_t total = cum[kSortClassBlock];
    while (true) {
        if (threadIdx.x == 0) ticket = g_atomic_add(lcnt + kSortTicketBlock, 1u);
        __syncthreads();
        const uint32_t t = (uint32_t)__builtin_amdgcn_readfirstlane((int)ticket);  // block-uniform
        __syncthreads();
        if (t >= total) break;
        int s = 0;
#pragma unroll
        for (int q = 1; q < kSortClassBlock; ++q) s += (t >= cum[q]) ? 1 : 0;
        uint32_t off = 0;
        int oc = 0, gs = 1;
#pragma unroll
        for (int q = 0; q < kSortClassBlock; ++q) {
            off = (q == s) ? cum[q] : off;
            oc = (q == s) ? order[q] : oc;
            gs = (q == s) ? gsz[q] : gs;
        }
        const int c = kSortClassWave + oc;
        const uint32_t cnt = min(lcnt[c], L.cap);
        const uint32_t first = (t - off) * (uint32_t)gs;
        const int nb = (int)min((uint32_t)gs, cnt - first);
        const gptr<const uint32_t> ents = glb((const uint32_t *)L.list) + (size_t)c * L.cap + first;
        switch (oc) {
        case 0: block_buckets<true, 2>(items, ents, nb, lds, dl, L.diag0); break;    // packed 2048
        case 1: block_buckets<true, 4>(items, ents, nb, lds, dl, L.diag0); break;    // packed 4096
        case 2: block_buckets<true, 8>(items, ents, nb, lds, dl, L.diag0); break;    // packed 8192
        case 3: block_buckets<true, 16>(items, ents, nb, lds, dl, L.diag0); break;   // packed 16384
        case 4: block_buckets<false, 2>(items, ents, nb, lds, dl, L.diag0); break;   // wide 1024
        case 5: block_buckets<false, 4>(items, ents, nb, lds, dl, L.diag0); break;   // wide 2048
        case 6: block_buckets<false, 8>(items, ents, nb, lds, dl, L.diag0); break;   // wide 4096
        default: block_buckets<false, 16>(items, ents, nb, lds, dl, L.diag0); break; // wide 8192
        }
        __syncthreads();
    }
    diag_lds_end<kSortBlockThreads>(L, dl);
}

// ----------------------------------------------------- global kernel --
// Buckets beyond the block classes: LSD radix sort in the bucket's own
// global-memory slice (ping-pong with the second composite array) -- packed
// words by their composite half, wide composites with their index array --
// then the block-wide segmentation with scratch taken from the free slices.
template <bool PK>
__global__ __launch_bounds__(kThreads) void k_sort_global(const MaskWork *__restrict__ items, SortLists L, int cls)
{
    using K = uint64_t;
    __shared__ SortScratch ss;
    const uint32_t cnt = min(glb(L.cnt)[cls], L.cap);
    for (uint32_t t = blockIdx.x; t < cnt; t += gridDim.x) {
        const uint32_t ent = glb(L.list)[(size_t)cls * L.cap + t];
        const MaskWork &W = items[ent >> kListBucketBits];
        const uint32_t bucket = ent & kListBucketMask;
        if (bucket >= (1u << W.B)) continue;
        const uint32_t base = glb(W.boff)[bucket];
        const uint32_t n = glb(W.boff)[bucket + 1] - base;
        const gptr<K> gc = glb(reinterpret_cast<K *>(W.comp)), gc2 = glb(reinterpret_cast<K *>(W.comp2));
        const gptr<uint32_t> ix = glb(W.idx), ix2 = glb(W.idx2);
        int which = 0;
        // packed words carry their index: the index arrays ride along unused
        block_radix_sort<K>(gc + base, ix + base, gc2 + base, ix2 + base, n, W.cb, ss, which, PK ? W.ib : 0);
        __syncthreads();
        const gptr<K> fk = (which ? gc2 : gc) + base;
        const gptr<uint32_t> fv = (which ? ix2 : ix) + base;
        const gptr<uint32_t> fr = (gptr<uint32_t>)(which ? gc : gc2);
        const gptr<uint32_t> fx = (which ? ix : ix2) + base;
        // scratch: this bucket's slice of the free composite array (2n words)
        block_segment(fk, fv, n, fr + 2 * (size_t)base, fr + 2 * (size_t)base + n, fx, W, base, ss.wsum, bucket, PK ? W.ib : 0);
        __syncthreads();
    }
}

// --------------------------------------------------------------- launchers --
hipError_t launch_bucket_scan(const MaskWork *items, int nitems, SortLists L, hipStream_t st)
{
    if (!nitems) return hipSuccess;
    hipLaunchKernelGGL(k_bucket_scan, dim3(nitems), dim3(kThreads), 0, st, items, L);
    return hipGetLastError();
}

hipError_t launch_sort_wave(const MaskWork *items, SortLists L, const SortGrid &g, hipStream_t st)
{
    if (g.wave_blocks)
        hipLaunchKernelGGL(k_sort_wave<false>, dim3(g.wave_blocks), dim3(kThreads), (size_t)L.ndiag * 4, st, items, L);
    return hipGetLastError();
}

hipError_t launch_sort_wave_big(const MaskWork *items, SortLists L, const SortGrid &g, hipStream_t st)
{
    if (g.wave_big_blocks)
        hipLaunchKernelGGL(k_sort_wave<true>, dim3(g.wave_big_blocks), dim3(kThreads), (size_t)L.ndiag * 4, st, items, L);
    return hipGetLastError();
}

hipError_t launch_sort_block(const MaskWork *items, SortLists L, const SortGrid &g, hipStream_t st)
{
    if (g.block_blocks)
        hipLaunchKernelGGL(k_sort_block, dim3(g.block_blocks), dim3(kSortBlockThreads), (size_t)L.ndiag * 4, st, items, L);
    return hipGetLastError();
}

hipError_t launch_sort_global(const MaskWork *items, SortLists L, const SortGrid &g, hipStream_t st)
{
    if (g.global_blocks_pk)
        hipLaunchKernelGGL(k_sort_global<true>, dim3(g.global_blocks_pk), dim3(kThreads), 0, st, items, L,
                           kSortClassWave + kSortClassBlock);
    if (g.global_blocks_wide)
        hipLaunchKernelGGL(k_sort_global<false>, dim3(g.global_blocks_wide), dim3(kThreads), 0, st, items, L,
                           kSortClassWave + kSortClassBlock + 1);
    return hipGetLastError();
}

}  // namespace gk
