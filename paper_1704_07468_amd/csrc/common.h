// Device-side data structures and block-level primitives of the gfx950
// gapped k-mer kernel library.  Wave size is 64 everywhere; blocks have
// kThreads = 256 threads (4 waves).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gk {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxRuns = 33;     // kept positions form at most min(g-m, m+1) <= 33 runs (g <= 64)
constexpr int kTile = 4096;      // g-mers per block in the partition scatter
constexpr int kScatterThreads = 512;  // its threads: 8 g-mers each, 8 waves per SIMD
constexpr int kCountTile = 16384;  // g-mers per 1024-thread block in the bucket count
constexpr int kCountThreads = 1024;
constexpr int kMaxBucketBits = 14;
// a sort-list entry is (mask in the chunk) << kListBucketBits | bucket
constexpr int kListBucketBits = kMaxBucketBits;
constexpr uint32_t kListBucketMask = (1u << kListBucketBits) - 1u;
constexpr int kMaxChunkMasks = 1 << (32 - kListBucketBits);

// Bucket size classes of the per-bucket sort: nine wave classes (packed
// composites 64..1024 g-mers, wide ones 64..512; the largest of each, packed
// 1024 and wide 512, in a second wave kernel with more LDS per wave), eight
// block classes (packed 2048..16384, wide 1024..8192) and two global-memory
// classes (packed, wide).
constexpr uint32_t kSortWaveMaxPk = 1024;
constexpr uint32_t kSortWaveMaxWide = 512;
constexpr uint32_t kSortBlockMaxPk = 16384;
constexpr uint32_t kSortBlockMaxWide = 8192;
constexpr int kSortClassWave = 9;
constexpr int kSortClassBlock = 8;
constexpr int kSortClasses = kSortClassWave + kSortClassBlock + 2;
constexpr int kSortTicketBlock = kSortClasses;  // counter slot of the block kernel's work tickets
constexpr int kSortCounters = 32;               // counter words per chunk

// Per-class lists of (mask << 12 | bucket) entries, cap entries per class,
// and their counters.
struct SortLists {
    uint32_t *cnt;   // [kSortCounters] zeroed before the scan
    uint32_t *list;  // [kSortClasses][cap]
    uint32_t cap;
    unsigned long long *stat;  // nullable: g-mers per kernel (wave, block, global) x (packed, wide)
    // the diagonal counters of the chunk's masks when they form one array of
    // at most kDiagLds words (a query batch): the sort kernels sum into LDS
    // and add each block's sums once at its end (ndiag = 0: direct atomics)
    uint32_t *diag0;
    uint32_t ndiag;
};
constexpr uint32_t kDiagLds = 1024;

// One set of removed positions ("mask"), as the runs of kept symbol fields:
// reduced = OR_r ((key >> src[r]) & (2^wid[r]-1)) << dst[r].  The kept
// symbols keep their order, first kept symbol most significant, so equal
// reduced keys <=> equal (g-m)-mers (Section 2.2, step 3).
struct MaskDesc {
    int32_t level;  // m
    int32_t nrun;
    // run i: bits [src, src + wid) of the key go to [dst, dst + wid) of the
    // reduced key; packed src | wid << 8 | dst << 16 in one word, so that a
    // block reads the table with scalar loads
    uint32_t run[kMaxRuns];
};

// int8 matrix-core path geometry: 128 x 128 output tiles, rows staged 64 at
// a time, a row split holding at most 65536 rows (65536 * 127^2 < 2^31 keeps
// its int32 partial sums exact).
constexpr int kDenseTile = 128;
constexpr int kDenseK = 64;
constexpr uint32_t kDenseSplitRows = 65536;
constexpr int kDenseMaxSplits = 8;  // row splits per output tile

// Per level of a job: the split partial tiles of its count-matrix products
// (P == nullptr when the level has none), added by the epilogue.
struct DenseRef {
    const int32_t *P;        // [upper tiles][S][128 * 128]
    const uint32_t *count;   // rows used (device counter)
    uint32_t cap;            // row capacity
    int32_t S, ntile;        // row splits; tiles per edge
};

// Per-dataset ("job") state.
struct JobDev {
    const int8_t *seqs;      // concatenated symbol codes
    const int64_t *seq_off;  // [N+1] symbol offset of each sequence
    const uint32_t *gstart;  // [N+1] first g-mer of each sequence
    int32_t N, sigma, g, k, M, b, sb;  // sb = bits of a sequence id
    uint32_t T;              // number of g-mers
    int64_t nsym;            // total symbols
    uint64_t *key;           // [T] packed g-mers, first symbol most significant; with
                             // kshift > 0 the sequence id sits above them (key >> kshift)
    int32_t kshift;          // g * b when g * b + sb <= 64 (and the keys are internal), else 0
    uint32_t *sid;           // [T] sequence of each g-mer
    int32_t *err;            // bit 0: a symbol outside [0, sigma); bit 1: excess list full
    int64_t *C;              // [M+1][N][N] cumulative profiles (upper triangle accumulated)
    int64_t *Kd;             // [N] unnormalised K diagonal
    const int64_t *coef;     // [(M+1)*(M+1)] C(g-j, m-j) at [m*(M+1)+j]
    const int64_t *hco;      // [M+1] C(g-m, k)
    const DenseRef *dref;    // [M+1] int8-path partials per level
    double *K_out;
    int64_t *Nm_out;
    int64_t *Cm_out;
};

// Direct-address grouping of a level whose reduced g-mers take at most
// kDirectMaxKeys values (sigma^(g-m) of them): no partition and no sort.  A
// position set's groups are indexed by the reduced g-mer itself (base-sigma
// digits, first kept symbol most significant), so every possible reduced
// g-mer is one row of the level's count matrix D, D[X][row] = how often
// sequence X holds it (Section 2.2 step 3: the groups of equal reduced
// g-mers and their per-sequence counts), and the level's whole C_m is D^T D
// on the matrix cores.  Counts above 127 are stored as 127; the excess is
// recorded and corrected exactly afterwards.
constexpr uint32_t kDirectMaxKeys = 16384;
constexpr int kDirectMasksPerBlock = 1;  // position sets of one level per block of the row writer (more measured slower)

struct DirectLevel {
    int8_t *D;         // [Ntile][stride] sequence-major counts (tiled_offset layout); rows [0, R) used
    uint32_t stride;   // bytes per sequence (R rounded up to 64)
    uint32_t R;        // rows: position sets of the level x Kp
    uint32_t Kp;       // rows per position set: sigma^(g-m) rounded up to 16
    int32_t job, level;
    int32_t nd;        // kept symbols, g - m
    int32_t b, sigma;  // symbol bits and alphabet size
    int32_t pow2;      // 1: sigma = 2^b, the row is the compacted key itself
};

// One position set of a directly addressed level.
struct DirectWork {
    MaskDesc md;
    int32_t dl;        // its DirectLevel
    uint32_t row0;     // first count-matrix row of this position set
    int32_t first;     // 1: the level's first position set (clears the level's C_m rows)
    int32_t last;      // 1: the level's last position set (zeroes the rows past R)
};

// Counts above 127 of directly addressed position sets: (row, sequence,
// count - 127, direct level) per entry.  Past cap entries the call is redone
// without direct addressing.
struct ExcessList {
    uint4 *ent;
    uint32_t *count;
    uint32_t cap;
};

// Per (job, mask) work of the partition sort and its outputs.
struct MaskWork {
    MaskDesc md;
    int32_t job;
    uint32_t T;
    int32_t N;   // sequences of the job
    int32_t w;   // bits of the reduced key
    int32_t B;   // bucket bits (top bits of the hashed reduced key)
    int32_t hb;  // remaining hash bits, w - B
    int32_t sb;  // sequence-id bits
    int32_t cb;  // composite sort bits, hb + sb
    int32_t ib;  // index bits of a packed word: ceil(log2(T + 1)), so no index field is all ones
    const uint64_t *key;
    const uint32_t *sid;
    uint32_t *bcnt;   // [2^B]
    uint32_t *boff;   // [2^B + 1]
    uint32_t *bcur;   // [2^B]
    uint64_t *comp;   // [T] composite (hash rest, sequence) of each bucketed g-mer; when
                      // cb + ib <= 64, packed with its g-mer index: composite << ib | index
    uint32_t *idx;    // [T] g-mer index of a wide composite
    uint64_t *comp2;  // [T] ping-pong buffers for buckets sorted in global memory
    uint32_t *idx2;   // [T]
    uint32_t *E;      // [T] run entries: sequence | count << sb, grouped, sequence-sorted
    uint2 *info;      // [T] per g-mer: (entry index, entries to group end) for run leaders
    // int8 matrix-core path for groups with many distinct sequences
    int8_t *D;         // level's count matrix, sequence-major, tiled: D[tiled_offset(sid, row, dstride)] (nullable)
    uint32_t *dcount;  // rows used
    uint32_t dcap;     // row capacity
    uint32_t dstride;  // bytes per sequence
    int32_t tau;       // min distinct sequences of a dense group (0 = off)
    int32_t inl;       // 1: a run two entries from its group end carries the
                       // last entry in its info instead of its own index
    int32_t i4;        // 1: 4-byte info records (pack_info4), 0: uint2 records
    int32_t kshift;    // > 0: each key carries its sequence id at this bit (the job's kshift)
    // resident tables (serving): per bucket its groups in hash-rest order
    uint4 *gtab;       // [T] (hash rest lo, hi, first entry, end entry) at bucket offset + group (nullable)
    uint32_t *bgrp;    // [2^B] groups per bucket
    uint32_t *diag;    // [N] sum over runs of count^2 per sequence, this level (nullable)
};

// Row accumulation work: rows of one job over a range of masks of one level.
// The masks' buffers lie mstride bytes apart (equal-size slices of the
// pool), so a mask's info and run-entry arrays are those of the first mask
// plus its index times mstride.
struct AccWork {
    int32_t job;
    int32_t mfirst;  // first MaskWork index
    int32_t nmask;
    int32_t level;
    int32_t Npad;    // LDS row stride (the slab width, a multiple of 64)
    int32_t first;   // 1: first work of its (job, level): store the row, else add
    int32_t slab, nslab;  // columns per block and blocks per row
    int32_t mstep;   // masks summed in the int32 LDS row between flushes (0: all)
    int32_t pad;
    int64_t mstride;
};

// --------------------------------------------------------------------------
// Global-memory pointers.  Pointers read from descriptors are generic, and
// generic (flat) accesses also count against the LDS counter, so every LDS
// wait after them waits for the global access too; kernels that mix LDS work
// with global accesses go through these.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ gptr<T> glb(T *p) { return (gptr<T>)p; }
template <typename T>
__device__ __forceinline__ T g_atomic_add(gptr<T> p, T v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// uint2 / uint4 records through global pointers (as plain words: the HIP
// vector classes cannot be assigned in another address space)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void st_u2(gptr<uint2> p, size_t i, uint32_t x, uint32_t y)
{
    ((gptr<uint64_t>)p)[i] = ((uint64_t)y << 32) | x;
}
__device__ __forceinline__ uint2 ld_u2(gptr<const uint2> p, size_t i)
{
    const uint64_t v = ((gptr<const uint64_t>)p)[i];
    return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
}
__device__ __forceinline__ void st_u4(gptr<uint4> p, size_t i, uint32_t a, uint32_t b, uint32_t c, uint32_t d)
{
    ((gptr<u32x4>)p)[i] = u32x4{a, b, c, d};
}

// Compact per-g-mer record of a run leader for the row accumulation (Gram
// calls with at most 2^21 g-mers and sequence ids of at most 12 bits), 4
// bytes instead of a uint2: bits 0-6 the entries from the run's own to its
// group end (127: the length is in the side array at the run's entry index),
// bit 7 set when the group's last run is carried inline, bits 8-10 the run's
// count (0: 8 or more, read from the run's entry), bits 11-31 the payload:
// the run's count when it is its group's last run, the last run's entry
// (sequence | count << sb) when inline, else the run's entry index.
// The records start zeroed (the partition clears them) and only nonzero ones
// are stored.  0: nothing beyond the g-mer's own diagonal term 1 -- not a run
// leader, or the last run of its group with count 1 (most g-mers of the
// sparse levels), whose self-pair 1 * 1 is that term.  A run summed on the
// matrix cores stores 128 | count << 8 (bits 0-6 zero): the product adds its
// count^2 to the diagonal, so the accumulation takes back the count's worth
// of unit terms.
// Run entries of the same calls are 16 bits: sequence | count << sb, the
// count field 0 when the count needs more than 16 - sb bits; the count is
// then in the escape half of the entry array (16-bit slot T + entry).
__device__ __forceinline__ void store_entry16(gptr<uint16_t> E16, uint32_t T, uint32_t e, uint32_t sid, uint32_t cnt, int sb)
{
    if (cnt < (1u << (16 - sb))) {
        E16[e] = (uint16_t)(sid | (cnt << sb));
    } else {
        E16[e] = (uint16_t)sid;
        E16[T + e] = (uint16_t)cnt;  // at most 65535 g-mers per sequence
    }
}

constexpr uint32_t kInfo4MaxT = 1u << 21;
__device__ __forceinline__ uint32_t pack_info4(uint32_t len, uint32_t cnt, uint32_t ei, bool inl, uint32_t last_entry,
                                               int sb, __attribute__((address_space(1))) uint32_t *lenx)
{
    if (len == 0) return 128u | (cnt << 8);  // count-matrix run (count <= 127)
    if (len == 1) return cnt == 1u ? 0u : (1u | (cnt << 11));
    if (inl && len == 2 && cnt <= 7u && (last_entry >> sb) < (1u << (21 - sb)))
        return 2u | (1u << 7) | (cnt << 8) | (last_entry << 11);
    uint32_t lf = len;
    if (len >= 127u) {
        lf = 127u;
        lenx[ei] = len;
    }
    return lf | ((cnt <= 7u ? cnt : 0u) << 8) | (ei << 11);
}

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << __lane_id()) - 1ull; }

__device__ __forceinline__ uint64_t bits_mask(int w) { return (w >= 64) ? ~0ull : ((1ull << w) - 1ull); }

// Bijection on w-bit integers (odd multiplies and right xor-shifts, each
// invertible modulo 2^w).  Equal inputs <=> equal outputs, and the top bits
// spread skewed key distributions evenly over the buckets.
__device__ __forceinline__ uint64_t mix_w(uint64_t x, int w)
{
    if (w <= 0) return 0;
    const uint64_t m = bits_mask(w);
    const int s = (w + 1) >> 1;
    x = (x * 0x9E3779B97F4A7C15ull) & m;
    x ^= x >> s;
    x = (x * 0xC2B2AE3D27D4EB4Full) & m;
    x ^= x >> s;
    return x;
}

__device__ __forceinline__ uint64_t compact_key(uint64_t key, const MaskDesc &md)
{
    uint64_t r = 0;
    for (int i = 0; i < md.nrun; ++i) {
        const uint32_t w = md.run[i];
        r |= ((key >> (w & 0xFF)) & bits_mask((int)((w >> 8) & 0xFF))) << (w >> 16);
    }
    return r;
}

// compact_key of Q keys at once: each run of the mask is read once for all
// of them (the run table is the same for the whole block).
template <int Q>
__device__ __forceinline__ void compact_keys(const uint64_t (&key)[Q], uint64_t (&r)[Q], const MaskDesc &md)
{
#pragma unroll
    for (int q = 0; q < Q; ++q) r[q] = 0;
    for (int i = 0; i < md.nrun; ++i) {
        const uint32_t w = md.run[i];
        const uint32_t src = w & 0xFF, dst = w >> 16;
        const uint64_t msk = bits_mask((int)((w >> 8) & 0xFF));
#pragma unroll
        for (int q = 0; q < Q; ++q) r[q] |= ((key[q] >> src) & msk) << dst;
    }
}

// int8 count matrices of the matrix-core products (one row of `stride`
// counts per sequence, stride a multiple of 64) are stored in tiles of 128
// sequences: columns [64 k, 64 k + 64) of a tile's sequences form one
// contiguous 8 KB block (sequence-major inside), and a tile's blocks follow
// in column order, so a product step reads each operand tile as one block.
// Sequence x, column c lies at this offset.
__device__ __forceinline__ size_t tiled_offset(uint32_t x, size_t c, size_t stride)
{
    return ((size_t)(x >> 7) * 128u) * stride + (c >> 6) * 8192u + (size_t)(x & 127u) * 64u + (c & 63u);
}

// Rows [r0, r1) of split s of at most S when R rows are used: whole 64-row
// steps, at least kDenseMinSplitRows rows per split, so that a level with
// few rows writes (and its epilogue reads) few partial tiles.
constexpr uint32_t kDenseMinSplitRows = 32768;
__device__ __forceinline__ void split_range(uint32_t R, int S, int s, uint32_t &r0, uint32_t &r1)
{
    const uint32_t used = max(1u, min((uint32_t)S, (R + kDenseMinSplitRows - 1) / kDenseMinSplitRows));
    const uint32_t per = ((R + used - 1) / used + kDenseK - 1) / kDenseK * kDenseK;
    r0 = min(R, per * (uint32_t)s);
    r1 = min(R, r0 + per);
}

// Splits of a level that hold rows (they come first).
__device__ __forceinline__ int dense_splits_used(const DenseRef &D)
{
    if (!D.P) return 0;
    const uint32_t R = min(*D.count, D.cap);
    int ns = 0;
    for (int s = 0; s < D.S; ++s) {
        uint32_t r0, r1;
        split_range(R, D.S, s, r0, r1);
        if (r0 < r1) ns = s + 1;
    }
    return ns;
}

// Offset of element (x, y) (tile-local, 0..127) in a 128 x 128 partial tile
// stored as sixteen contiguous 32 x 32 sub-tiles, the epilogue's tile.
__device__ __forceinline__ uint32_t dense_tile_offset(int x, int y)
{
    return (uint32_t)(((x >> 5) * 4 + (y >> 5)) * 1024 + (x & 31) * 32 + (y & 31));
}

// The int8-path part of C_m[x][y] (x <= y): the sum of the used splits'
// partial tiles.
__device__ __forceinline__ int64_t dense_part(const DenseRef &D, int ns, int x, int y)
{
    const int I = x / kDenseTile, Jt = y / kDenseTile;
    const int f = I * D.ntile - (I * (I - 1)) / 2 + (Jt - I);
    const size_t e = dense_tile_offset(x % kDenseTile, y % kDenseTile);
    const gptr<const int32_t> p = glb((const int32_t *)D.P) + (size_t)f * D.S * (kDenseTile * kDenseTile) + e;
    int64_t v = 0;
#pragma unroll
    for (int s = 0; s < kDenseMaxSplits; ++s)  // independent loads, issued together
        if (s < ns) v += p[(size_t)s * (kDenseTile * kDenseTile)];
    return v;
}

// Index i with prefix[i] <= v < prefix[i+1]; prefix has n+1 entries.
__device__ __forceinline__ int find_item(const uint32_t *prefix, int n, uint32_t v)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x)
{
    // within each row of 16 lanes: shifted adds (row_shr:1, 2, 4, 8; a lane
    // shifted in from outside the row adds 0)
    x += __builtin_amdgcn_update_dpp(0u, x, 0x111, 0xF, 0xF, false);
    x += __builtin_amdgcn_update_dpp(0u, x, 0x112, 0xF, 0xF, false);
    x += __builtin_amdgcn_update_dpp(0u, x, 0x114, 0xF, 0xF, false);
    x += __builtin_amdgcn_update_dpp(0u, x, 0x118, 0xF, 0xF, false);
    // then the totals of the rows below
    const uint32_t r0 = __builtin_amdgcn_readlane(x, 15);
    const uint32_t r1 = r0 + __builtin_amdgcn_readlane(x, 31);
    const uint32_t r2 = r1 + __builtin_amdgcn_readlane(x, 47);
    const int row = __lane_id() >> 4;
    return x + (row == 0 ? 0u : row == 1 ? r0 : row == 2 ? r1 : r2);
}

// Set bits of m below this lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Block-wide exclusive scan of one value per thread (kThreads threads).
// Contains two barriers; every thread of the block must call it.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *wsum, uint32_t *total)
{
    const uint32_t inc = wave_incl_scan(v);
    const int wid = threadIdx.x >> 6;
    if (__lane_id() == 63) wsum[wid] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const uint32_t s = wsum[w];
        pre += (w < wid) ? s : 0u;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return pre + inc - v;
}

struct SortScratch {
    uint32_t hist[256];
    uint32_t base[256];
    uint32_t wcnt[kWaves][256];
    uint32_t wsum[kWaves];
};

constexpr int kE = 4;  // elements per thread per round of the radix passes and the segmentation

// Stable LSD radix sort of n (key, value) pairs by key bits [shift0,
// shift0 + bits), 8 bits per pass, ping-ponging between (k0,v0) and (k1,v1).  A pass is
// an LDS digit histogram, a block scan of it, and rounds of 1024 elements: in
// each round every wave ranks 4 consecutive groups of 64 elements by digit
// with ballots -- the lanes holding the same digit form a ballot mask, a
// lane's rank is the population count of that mask below it, and the lowest
// lane of the mask advances the wave's running count of the digit with one
// LDS atomic whose old value it shares by shuffle -- then the waves' counts
// are combined.  Passes whose digit is the same for every element are
// skipped.  `which` says where the data is on entry (0: k0/v0) and is updated.
template <typename K, typename KP, typename VP>
__device__ __forceinline__ void block_radix_sort(KP k0, VP v0, KP k1, VP v1, uint32_t n, int bits,
                                                 SortScratch &s, int &which, int shift0 = 0)
{
    const int tid = threadIdx.x, wid = tid >> 6, lane = __lane_id();
    const uint64_t lt = lanemask_lt();
    for (int shift = shift0; shift < shift0 + bits; shift += 8) {
        KP sk = which ? k1 : k0;
        VP sv = which ? v1 : v0;
        KP dk = which ? k0 : k1;
        VP dv = which ? v0 : v1;
        s.hist[tid] = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) s.wcnt[w][tid] = 0;
        __syncthreads();
        for (uint32_t i = tid; i < n; i += kThreads)
            atomicAdd(&s.hist[(uint32_t)(sk[i] >> shift) & 255u], 1u);
        __syncthreads();
        const uint32_t c = s.hist[tid];
        uint32_t tot;
        const uint32_t ex = block_excl_scan(c, s.wsum, &tot);
        if (__syncthreads_or(c == n)) continue;  // one digit only: order unchanged
        s.base[tid] = ex;
        __syncthreads();
        for (uint32_t r0 = 0; r0 < n; r0 += kThreads * kE) {
            K kk[kE];
            uint32_t vv[kE], dd[kE], pp[kE];
#pragma unroll
            for (int e = 0; e < kE; ++e) {
                const uint32_t i = r0 + (uint32_t)(wid * 64 * kE + e * 64 + lane);
                const bool ok = i < n;
                kk[e] = ok ? (K)sk[i] : (K)0;
                vv[e] = ok ? (uint32_t)sv[i] : 0u;
                dd[e] = ok ? ((uint32_t)(kk[e] >> shift) & 255u) : 256u;
                uint64_t peers = __ballot(ok);
#pragma unroll
                for (int bb = 0; bb < 8; ++bb) {
                    const uint64_t m = __ballot((dd[e] >> bb) & 1u);
                    peers &= ((dd[e] >> bb) & 1u) ? m : ~m;
                }
                const uint32_t rank = __popcll(peers & lt);
                uint32_t old = 0;
                if (ok && rank == 0) old = atomicAdd(&s.wcnt[wid][dd[e]], (uint32_t)__popcll(peers));
                const int leader = peers ? (__ffsll((long long)peers) - 1) : lane;
                old = __shfl(old, leader, 64);
                pp[e] = old + rank;
            }
            __syncthreads();
#pragma unroll
            for (int e = 0; e < kE; ++e) {
                if (dd[e] < 256u) {
                    uint32_t off = s.base[dd[e]];
                    for (int w = 0; w < wid; ++w) off += s.wcnt[w][dd[e]];
                    dk[off + pp[e]] = kk[e];
                    dv[off + pp[e]] = vv[e];
                }
            }
            __syncthreads();
            uint32_t add = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                add += s.wcnt[w][tid];
                s.wcnt[w][tid] = 0;
            }
            s.base[tid] += add;
            __syncthreads();
        }
        which ^= 1;
    }
}

// Largest i in [0, n) with a[i] <= v (a ascending, a[0] <= v).
template <typename UP>
__device__ __forceinline__ uint32_t last_le(UP a, uint32_t n, uint32_t v)
{
    uint32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (a[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Segment a bucket sorted by (hash rest, sequence): runs of equal composite
// are one (reduced g-mer, sequence) pair; groups of equal hash rest are one
// reduced g-mer.  Writes one run entry (sequence | count << sb) per run into
// E[ebase + r] -- so each group's entries are contiguous and sequence-sorted
// -- and for every g-mer its info: the leader of a run (its first element)
// gets (entry index, entries left to the group end), every other g-mer
// (0, 0).  Groups with at least tau distinct sequences and counts <= 127
// become rows of the int8 matrix-core path instead (info length 0).
// rpos, gsr, gaux: scratch of n entries each.  Runs and groups are found in
// rounds of 1024 elements, 4 consecutive ones per thread, with one block scan
// per round for each.
// With W.gtab set, the bucket's groups are also listed (hash rest, first
// entry, end entry) at gtab[ebase + group] and their number at
// bgrp[bucket]; with W.diag set, every run adds count^2 to its sequence's
// diagonal counter (the self-pairs of Algorithm 1's countAndUpdate).
template <typename KP, typename VP, typename UP>
__device__ __forceinline__ void block_segment(KP fk, VP fv, uint32_t n, UP rpos, UP gsr, UP gaux,
                                              const MaskWork &W, uint32_t ebase, uint32_t *wsum, uint32_t bucket,
                                              int cshift)
{
    // cshift = 32: fk holds packed words (composite << 32 | g-mer index)
    auto comp = [&](uint32_t i) -> uint64_t { return (uint64_t)fk[i] >> cshift; };
    auto gidx = [&](uint32_t i) -> uint32_t {
        return cshift ? (uint32_t)((uint64_t)fk[i] & bits_mask(cshift)) : (uint32_t)fv[i];
    };
    const gptr<uint32_t> E = glb(W.E);
    const gptr<uint2> info = glb(W.info);
    const gptr<int8_t> D = glb(W.D);
    const int tid = threadIdx.x;
    const int sb = W.sb;
    const uint64_t sidmask = bits_mask(sb);
    uint32_t R = 0, G = 0;
    for (uint32_t r0 = 0; r0 < n; r0 += kThreads * kE) {
        const uint32_t i0 = r0 + (uint32_t)tid * kE;
        uint32_t rsf = 0, gsf = 0;  // bit e: element i0+e starts a run / a group
        uint64_t prev = (i0 > 0 && i0 <= n) ? comp(i0 - 1) : 0ull;
#pragma unroll
        for (int e = 0; e < kE; ++e) {
            const uint32_t i = i0 + e;
            if (i < n) {
                const uint64_t cur = comp(i);
                if (i == 0 || cur != prev) rsf |= 1u << e;
                if (i == 0 || (cur >> sb) != (prev >> sb)) gsf |= 1u << e;
                prev = cur;
            }
        }
        uint32_t rtot, gtot;
        uint32_t rx = block_excl_scan((uint32_t)__popc(rsf), wsum, &rtot);
        uint32_t gx = block_excl_scan((uint32_t)__popc(gsf), wsum, &gtot);
#pragma unroll
        for (int e = 0; e < kE; ++e) {
            if (gsf & (1u << e)) gsr[G + gx++] = R + rx;
            if (rsf & (1u << e)) rpos[R + rx++] = i0 + e;
        }
        R += rtot;
        G += gtot;
    }
    __syncthreads();
    const bool dense_on = (W.tau > 0) && (W.D != nullptr);
    if (dense_on) {
        for (uint32_t gi = tid; gi < G; gi += kThreads) gaux[gi] = 0;
        __syncthreads();
        for (uint32_t r = tid; r < R; r += kThreads) {
            const uint32_t pe = (r + 1 < R) ? rpos[r + 1] : n;
            __hip_atomic_fetch_max(&gaux[last_le(gsr, G, r)], pe - rpos[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        for (uint32_t gi = tid; gi < G; gi += kThreads) {
            const uint32_t re = (gi + 1 < G) ? gsr[gi + 1] : R;
            uint32_t row = 0xFFFFFFFFu;
            if (re - gsr[gi] >= (uint32_t)W.tau && gaux[gi] <= 127u) {
                row = g_atomic_add(glb(W.dcount), 1u);
                if (row >= W.dcap) row = 0xFFFFFFFFu;
            }
            gaux[gi] = row;
        }
        __syncthreads();
    }
    for (uint32_t r = tid; r < R; r += kThreads) {
        const uint32_t p = rpos[r];
        const uint32_t pe = (r + 1 < R) ? rpos[r + 1] : n;
        const uint32_t cnt = pe - p;
        const uint32_t sid = (uint32_t)(comp(p) & sidmask);
        const uint32_t gi = last_le(gsr, G, r);
        const uint32_t re = (gi + 1 < G) ? gsr[gi + 1] : R;
        const uint32_t e = ebase + r;
        if (W.i4) store_entry16(glb((uint16_t *)W.E), W.T, e, sid, cnt, sb);
        else E[e] = sid | (cnt << sb);
        uint32_t len = re - r;
        if (dense_on) {
            const uint32_t row = gaux[gi];
            if (row != 0xFFFFFFFFu) {
                D[tiled_offset(sid, row, W.dstride)] = (int8_t)cnt;
                len = 0;
            }
        }
        uint32_t x = e;
        if (W.inl && len == 2) {  // the group's last run, inline
            const uint32_t p1 = rpos[r + 1];
            const uint32_t c1 = ((r + 2 < R) ? rpos[r + 2] : n) - p1;
            x = (uint32_t)(comp(p1) & sidmask) | (c1 << sb);
        }
        if (W.i4) {
            const uint32_t rec = pack_info4(len, cnt, e, W.inl && len == 2, x, sb, (gptr<uint32_t>)info + W.T);
            if (rec) ((gptr<uint32_t>)info)[gidx(p)] = rec;
        } else {
            // y: entries to the group end in the low sb+1 bits, the run count above
            st_u2(info, gidx(p), x, len ? (len | (cnt << (sb + 1))) : 0u);
        }
    }
    if (!W.i4)  // (4-byte records start zeroed)
        for (uint32_t i = tid; i < n; i += kThreads)
            if (i > 0 && comp(i) == comp(i - 1)) st_u2(info, gidx(i), 0u, 0u);
    if (W.gtab) {
        for (uint32_t gi = tid; gi < G; gi += kThreads) {
            const uint32_t r0 = gsr[gi];
            const uint32_t r1 = (gi + 1 < G) ? gsr[gi + 1] : R;
            const uint64_t hr = comp(rpos[r0]) >> sb;
            st_u4(glb(W.gtab), ebase + gi, (uint32_t)hr, (uint32_t)(hr >> 32), ebase + r0, ebase + r1);
        }
        if (tid == 0) glb(W.bgrp)[bucket] = G;
    }
    if (W.diag) {
        for (uint32_t r = tid; r < R; r += kThreads) {
            const uint32_t p = rpos[r];
            const uint32_t cnt = ((r + 1 < R) ? rpos[r + 1] : n) - p;
            g_atomic_add(glb(W.diag) + (uint32_t)(comp(p) & sidmask), cnt * cnt);
        }
    }
}

// ----------------------------------------------------------- wave level --
// The same sort and segmentation done by one wave on its own bucket, with no
// block barrier: LDS accesses of one wave are ordered, and wave_sync keeps
// the compiler from moving them across the phase boundaries.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Block -> (item, block within item): arithmetic when every item has the
// same number of blocks, else a search of the per-item block prefix.
// Block b of a grid of nb blocks runs on XCD b % 8 (blocks are dealt round-
// robin to the 8 XCDs).  xcd_order(b, nb) renumbers the blocks so that each
// XCD runs one contiguous range of the work: blocks writing the same region
// then share one L2, where their partial-line writes merge.
__device__ __forceinline__ uint32_t xcd_order(uint32_t b, uint32_t nb)
{
    const uint32_t q = nb / 8, rem = nb % 8, x = b % 8;
    return x * q + min(x, rem) + b / 8;
}

__device__ __forceinline__ void map_block(const uint32_t *prefix, int n, uint32_t uniform, uint32_t bid, int &item,
                                          uint32_t &sub)
{
    if (uniform) {
        item = (int)(bid / uniform);
        sub = bid - (uint32_t)item * uniform;
    } else {
        item = find_item(prefix, n, bid);
        sub = bid - prefix[item];
    }
}

}  // namespace gk
