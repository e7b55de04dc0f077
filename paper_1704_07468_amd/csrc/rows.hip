// gfx950 kernels of the serving path: kernel rows of query sequences against
// a resident set kept as per-position-set group tables.
//
// For a query q, a level m and one of its position sets, every g-mer of q is
// reduced, hashed into the resident table's bucket, and its group (the
// resident sequences holding the same reduced g-mer, with counts) found by a
// binary search of the bucket's hash-ordered group list.  Each entry
// (sequence sv, count c) of the group adds c to row[sv]: summed over the
// g-mers of q this is count_q * count_sv per reduced g-mer, i.e. the q-by-sv
// entries of Algorithm 1's countAndUpdate.  Rows of C_m then go through
// Eq. 9, Eq. 7, the cosine normalisation and Eq. 1's decision value.
#include <algorithm>

#include "common.h"
#include "launch.h"

namespace gk {

struct ResMask {
    MaskDesc md;
    int32_t w, B, hb, sb;
    const uint32_t *boff;  // [2^B + 1] first entry of each bucket
    const uint32_t *bgrp;  // [2^B] groups per bucket
    const uint32_t *E;     // run entries: sequence | count << sb
    const uint4 *gtab;     // groups (hash rest lo, hi, first entry, end entry)
};

struct RowsArgs {
    const uint64_t *qkey;      // query g-mers, packed
    const uint32_t *qgstart;   // [nq + 1]
    int32_t nq, M, nsv, slab;  // SVs per block (one LDS row slab)
    int32_t nslab, mchunk;     // SV slabs; position sets per block
    const ResMask *rm;
    const int32_t *lev_first;  // first mask of each level
    const int32_t *lev_count;
    uint32_t *C;               // [M+1][nq][nsv], zeroed; blocks add their partial rows
    unsigned long long *updates;  // nullable (profiling): pair updates, spread over 256 slots
    int32_t dense_level;       // level joined on the matrix cores (-1: none) ...
    const uint32_t *qflag;     // ... except for the queries flagged here
};

__device__ __forceinline__ void wave_sync_rows()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// First index in E[a, b) whose sequence id is >= s (entries sequence-sorted,
// ids below nsv).  A long range is first narrowed around where s would fall
// if its ids were spread evenly (two probes), then binary-searched.
__device__ __forceinline__ uint32_t lower_sid(gptr<const uint32_t> E, uint32_t a, uint32_t b, uint32_t s, uint32_t sidmask,
                                              uint32_t nsv)
{
    if (b - a > 32) {
        constexpr uint32_t w = 8;
        const uint32_t gs = a + (uint32_t)(((uint64_t)(b - a) * s) / nsv);
        const uint32_t l = gs > a + w ? gs - w : a, r = min(b, gs + w);
        if ((E[l] & sidmask) >= s) {
            b = l + 1;  // the answer is at most l
        } else {
            a = l + 1;
            if (r < b && (E[r - 1] & sidmask) < s) a = r;  // at least r
            else b = r;                                      // in (l, r)
        }
    }
    while (a < b) {
        const uint32_t mid = (a + b) >> 1;
        if ((E[mid] & sidmask) < s) a = mid + 1; else b = mid;
    }
    return a;
}

// One block per (level, chunk of the level's position sets, query, SV slab),
// heavy levels first: the block's partial row lives in LDS and is added into
// C at the end (integer additions, so the sum does not depend on the order).
constexpr int kRowsWindow = 1024;  // updates per window: sixteen gathers in flight per lane
constexpr int kRowsU = kRowsWindow / 64;
__global__ __launch_bounds__(kThreads) void k_rows_accumulate(RowsArgs A)
{
    extern __shared__ uint32_t acc[];
    __shared__ uint64_t tbase[kWaves][64];  // per group range: entry address - 4 * its start in the sequence
    __shared__ uint32_t mark[kWaves][kRowsWindow / 32];  // range starts in the current window, one bit each
    const int per_item = A.nq * A.nslab;
    int idx = (int)(blockIdx.x / per_item);
    const int rem = (int)(blockIdx.x % per_item);
    const int q = rem / A.nslab, sl = rem % A.nslab;
    // item -> (level, first position set of the chunk, position sets)
    int level = 0, m0 = 0, mc = 0;
    for (int l = A.M; l >= 0; --l) {
        const int cnt = A.lev_count[l];
        const int nch = (cnt + A.mchunk - 1) / A.mchunk;
        if (idx < nch) {
            level = l;
            m0 = idx * A.mchunk;
            mc = min(A.mchunk, cnt - m0);
            break;
        }
        idx -= nch;
    }
    if (mc <= 0) return;
    if (level == A.dense_level && !A.qflag[q]) return;  // on the matrix cores
    const int s0 = sl * A.slab, s1 = min(A.nsv, s0 + A.slab);
    const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    for (int i = tid; i < s1 - s0; i += kThreads) acc[i] = 0;
    if (lane < kRowsWindow / 32) mark[wid][lane] = 0;
    uint32_t *const accy = acc - s0;  // SV sv at accy[sv]
    __syncthreads();
    const uint32_t t0 = A.qgstart[q];
    const uint32_t ng = A.qgstart[q + 1] - t0;
    const uint32_t total = ng * (uint32_t)mc;
    const ResMask *rm = A.rm + A.lev_first[level] + m0;
    const int sb = rm[0].sb;
    const uint32_t sidmask = (uint32_t)bits_mask(sb);
    unsigned long long wupd = 0;  // the wave's gathered pair updates (profiling count)
    for (uint32_t c0 = (uint32_t)wid * 64; c0 < total; c0 += kThreads) {
        const uint32_t it = c0 + lane;
        uint32_t len = 0;
        uint64_t ebase = 0;
        if (it < total) {
            const uint32_t s = it / ng;
            const ResMask &R = rm[s];
            const uint64_t h = mix_w(compact_key(glb(A.qkey)[t0 + (it - s * ng)], R.md), R.w);
            const uint32_t b = (uint32_t)(R.hb >= 64 ? 0 : (h >> R.hb));
            const uint64_t hr = h & bits_mask(R.hb);
            const gptr<const u32x4> gtab = (gptr<const u32x4>)glb(R.gtab);
            const uint32_t g0 = glb(R.boff)[b], g1 = g0 + glb(R.bgrp)[b];
            uint32_t lo = g0, hi = g1;
            while (lo < hi) {  // first group with hash rest >= hr
                const uint32_t mid = (lo + hi) >> 1;
                const u32x4 gm = gtab[mid];
                if ((((uint64_t)gm.y << 32) | gm.x) < hr) lo = mid + 1; else hi = mid;
            }
            if (lo < g1) {
                const u32x4 gm = gtab[lo];
                if ((((uint64_t)gm.y << 32) | gm.x) == hr) {
                    uint32_t e0 = gm.z, e1 = gm.w;
                    // the slab's part of the group (the first slab starts
                    // at the group's start, the last ends at its end)
                    if (s0 > 0) e0 = lower_sid(glb(R.E), e0, e1, (uint32_t)s0, sidmask, (uint32_t)A.nsv);
                    if (s1 < A.nsv) e1 = lower_sid(glb(R.E), e0, e1, (uint32_t)s1, sidmask, (uint32_t)A.nsv);
                    len = e1 - e0;
                    ebase = reinterpret_cast<uint64_t>(R.E + e0);
                }
            }
        }
        // the chunk's entry ranges end to end, walked kRowsWindow updates at a
        // time; each update finds its range from a ballot of the range-start marks
        const uint32_t inc = wave_incl_scan(len);
        const uint32_t work = __builtin_amdgcn_readlane(inc, 63);
        if (work == 0) continue;  // wave-uniform
        wupd += work;
        const uint32_t start = inc - len;
        const uint64_t nz = __ballot(len > 0);
        if (len > 0) tbase[wid][lanes_below(nz)] = ebase - 4ull * start;
        uint32_t done = 0;  // ranges started before the window
#pragma unroll 1
        for (uint32_t w = 0; w < work; w += kRowsWindow) {
            const bool here = len > 0 && start >= w && start < w + kRowsWindow;
            if (here) atomicOr(&mark[wid][(start - w) >> 5], 1u << ((start - w) & 31u));
            wave_sync_rows();
            uint64_t st[kRowsU];
#pragma unroll
            for (int u = 0; u < kRowsU; ++u) st[u] = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)mark[wid][2 * u + 1]) << 32) |
                        (uint32_t)__builtin_amdgcn_readfirstlane((int)mark[wid][2 * u]);  // wave-uniform
            wave_sync_rows();
            if (lane < kRowsWindow / 32) mark[wid][lane] = 0;
            // A position past the end (last window only) has k = the last
            // range, so clamping it to work - 1 re-reads that range's last
            // entry: every load is valid and none waits on a branch.
            uint32_t ent[kRowsU];
#pragma unroll
            for (int u = 0; u < kRowsU; ++u) {
                const uint32_t k = done + lanes_below(st[u]) + (uint32_t)((st[u] >> lane) & 1ull) - 1u;
                done += (uint32_t)__popcll(st[u]);
                const uint32_t p = min(w + 64u * u + (uint32_t)lane, work - 1u);
                ent[u] = *(gptr<const uint32_t>)(tbase[wid][k] + 4ull * p);
            }
#pragma unroll
            for (int u = 0; u < kRowsU; ++u) {
                const uint32_t p = w + 64u * u + (uint32_t)lane;
                if (p < work) atomicAdd(&accy[ent[u] & sidmask], ent[u] >> sb);
            }
        }
        wave_sync_rows();
    }
    if (A.updates && lane == 0 && wupd) atomicAdd(A.updates + (blockIdx.x & 255u), wupd);
    __syncthreads();
    const gptr<uint32_t> crow = glb(A.C) + ((size_t)level * A.nq + q) * A.nsv;
    for (int sv = s0 + tid; sv < s1; sv += kThreads) {
        const uint32_t v = acc[sv - s0];
        if (v) g_atomic_add(crow + sv, v);
    }
}

// Diagonal counters of the queries: for each query q and position set of
// level m, the sum over its reduced g-mers u of count_q(u)^2 (the self-pairs
// of Algorithm 1's countAndUpdate), added into diag[m][q].  One block per
// (query, group of position sets); per set, a histogram of the query's
// reduced g-mers in LDS: indexed by the reduced g-mer itself when its width
// fits the table, else an open-addressing table keyed by its (bijective)
// hash.  The table has at least twice as many slots as the query has g-mers.
struct QDiagArgs {
    const uint64_t *qkey;     // query g-mers, packed
    const uint32_t *qgstart;  // [nq + 1]
    int32_t nq, nmask, mpb;   // queries, position sets, sets per block
    int32_t tbits;            // table slots: 1 << tbits
    const ResMask *rm;        // the resident set's position sets (level order)
    uint32_t *diag;           // [M+1][nq], zeroed
};

__global__ __launch_bounds__(kThreads) void k_query_diag(QDiagArgs A)
{
    extern __shared__ uint64_t qtab[];  // [slots] hashed keys, then [slots] counts
    __shared__ uint32_t wsum[kWaves];
    const uint32_t slots = 1u << A.tbits;
    uint64_t *tk = qtab;
    uint32_t *tc = reinterpret_cast<uint32_t *>(qtab + slots);
    const int nch = (A.nmask + A.mpb - 1) / A.mpb;
    const int q = (int)(blockIdx.x / (unsigned)nch), ch = (int)(blockIdx.x % (unsigned)nch);
    const uint32_t t0 = A.qgstart[q], ng = A.qgstart[q + 1] - t0;
    if (ng == 0) return;  // no g-mers: nothing to add
    const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    const gptr<const uint64_t> key = glb(A.qkey) + t0;
    const int s1 = min(A.nmask, (ch + 1) * A.mpb);
#pragma unroll 1
    for (int s = ch * A.mpb; s < s1; ++s) {
        const ResMask &R = A.rm[s];
        const MaskDesc md = R.md;
        const int w = R.w;
        const bool direct = w <= A.tbits;  // reduced g-mers index the table
        for (uint32_t i = tid; i < slots; i += kThreads) {
            tc[i] = 0;
            if (!direct) tk[i] = ~0ull;  // empty (a hash of w < 64 bits is never all ones)
        }
        __syncthreads();
        for (uint32_t t = tid; t < ng; t += kThreads) {
            const uint64_t rk = compact_key(key[t], md);
            if (direct) {
                atomicAdd(&tc[(uint32_t)rk], 1u);
            } else {
                const uint64_t h = mix_w(rk, w);
                uint32_t slot = (uint32_t)h & (slots - 1u);
                while (true) {  // at most half the slots are taken: a free one is reached
                    const uint64_t prev = atomicCAS((unsigned long long *)&tk[slot], ~0ull, (unsigned long long)h);
                    if (prev == ~0ull || prev == h) break;
                    slot = (slot + 1u) & (slots - 1u);
                }
                atomicAdd(&tc[slot], 1u);
            }
        }
        __syncthreads();
        uint32_t sq = 0;
        for (uint32_t i = tid; i < slots; i += kThreads) {
            const uint32_t c = tc[i];
            sq += c * c;
        }
        sq = wave_incl_scan(sq);
        if (lane == 63) wsum[wid] = sq;
        __syncthreads();
        if (tid == 0) {
            uint32_t tot = 0;
            for (int i = 0; i < kWaves; ++i) tot += wsum[i];
            if (tot) g_atomic_add(glb(A.diag) + (size_t)md.level * A.nq + q, tot);
        }
        __syncthreads();  // the table and the sums are reused by the next set
    }
}

hipError_t launch_query_diag(const uint64_t *qkey, const uint32_t *qgstart, int nq, int nmask, int tbits, const void *rm,
                             uint32_t *diag, hipStream_t st)
{
    if (nq <= 0 || nmask <= 0) return hipSuccess;
    constexpr int mpb = 4;
    QDiagArgs a{qkey, qgstart, nq, nmask, mpb, tbits, reinterpret_cast<const ResMask *>(rm), diag};
    const unsigned nb = (unsigned)((size_t)nq * (size_t)((nmask + mpb - 1) / mpb));
    hipLaunchKernelGGL(k_query_diag, dim3(nb), dim3(kThreads), (size_t)12u << tbits, st, a);
    return hipGetLastError();
}

// ------------------------------------------------------ dense top level --
// A level whose reduced g-mers index at most 4096 values per position set can
// be joined on the matrix cores instead: count rows Q (queries) and D
// (resident sequences), one column per (position set, reduced g-mer) of the
// level, int8 counts; the level's C rows are Q D^T (the same sum over groups
// of count_q * count_sv as Algorithm 1's countAndUpdate).  A count above 127
// is clipped and flags its sequence: a flagged resident set does not use this
// path, a flagged query takes the level through the sparse walk instead.

// One block per (sequence, 8 position sets of the level): an LDS histogram of
// the sequence's reduced g-mers per set, written as its 2^w-byte segment of
// the count row (16-byte stores).
constexpr int kCountRowSets = 8;
__global__ __launch_bounds__(kThreads) void k_count_rows(const uint64_t *__restrict__ key,
                                                         const uint32_t *__restrict__ gstart, int nseq,
                                                         const ResMask *__restrict__ rm, int nset, int w,
                                                         int8_t *__restrict__ out, size_t stride,
                                                         uint32_t *__restrict__ flag)
{
    extern __shared__ uint32_t hist[];
    const uint32_t bins = 1u << w;
    const int nch = (nset + kCountRowSets - 1) / kCountRowSets;
    const int x = (int)(blockIdx.x / (unsigned)nch), ch = (int)(blockIdx.x % (unsigned)nch);
    const uint32_t t0 = gstart[x], t1 = gstart[x + 1];
    const int tid = threadIdx.x;
    const gptr<const uint64_t> gk = glb(key);
    bool over = false;
    const int s1 = min(nset, (ch + 1) * kCountRowSets);
#pragma unroll 1
    for (int s = ch * kCountRowSets; s < s1; ++s) {
        const MaskDesc md = rm[s].md;
        for (uint32_t i = tid; i < bins; i += kThreads) hist[i] = 0;
        __syncthreads();
        for (uint32_t t = t0 + tid; t < t1; t += kThreads) atomicAdd(&hist[(uint32_t)compact_key(gk[t], md)], 1u);
        __syncthreads();
        for (uint32_t i = (uint32_t)tid * 16u; i < bins; i += kThreads * 16u) {
            uint32_t wv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t v = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    uint32_t c = hist[i + (uint32_t)(q * 4 + b)];
                    if (c > 127u) {
                        c = 127u;
                        over = true;
                    }
                    v |= c << (8 * b);
                }
                wv[q] = v;
            }
            *(gptr<u32x4>)(glb(out) + tiled_offset((uint32_t)x, (size_t)s * bins + i, stride)) = u32x4{wv[0], wv[1], wv[2], wv[3]};
        }
        __syncthreads();  // the histogram is reused by the next set
    }
    if (over) atomicOr(flag + x, 1u);
}

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
constexpr int kGemmBN = 128;  // resident sequences per block
constexpr int kGemmBK = 64;   // count columns per step
constexpr int kGemmRow = kGemmBK + 16;  // padded LDS row (80 bytes: 16-byte reads without conflicts)
constexpr int kGemmNT = kGemmBN / 32;   // MFMA column tiles per wave

struct RowsGemmArgs {
    const int8_t *Q;         // [nq_pad][stride] query count rows (tiled_offset layout)
    const int8_t *D;         // [nsv_pad][stride] resident count rows (tiled)
    size_t stride;           // bytes per row (a multiple of kGemmBK)
    int32_t nq, nsv;         // real rows
    int32_t ntq, ntsv, S;    // query tiles, sequence tiles, column splits
    const uint32_t *qflag;   // [nq] 1: the query takes the sparse walk for this level
    uint32_t *C;             // [nq][nsv] the level's C rows (added to)
};

// v_mfma_i32_32x32x32_i8 layout as in the Gram products: lane l supplies row
// (l % 32) and 16 consecutive columns from 16 * (l / 32); accumulator v of
// lane l is element (8 (v / 4) + 4 (l / 32) + v % 4, l % 32).  One block =
// BM queries (256, or 128 for smaller batches) x 128 resident sequences x
// one split of the columns; blocks are ordered split-major so that the
// blocks running together share the query slab in L2 while every resident
// row is streamed from HBM once per query tile, in 8 KB pieces of the tiled
// layout.  Wave w computes queries
// [w BM/4, (w + 1) BM/4) as (BM/128) x 4 MFMA tiles; slabs are
// double-buffered through LDS with 16-byte loads, two steps in flight.
template <int BM>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_rows_gemm(RowsGemmArgs A)
{
    constexpr int WR = BM / kWaves;  // query rows per wave
    constexpr int MT = WR / 32;      // MFMA row tiles per wave
    __shared__ __attribute__((aligned(16))) int8_t sA[2][BM][kGemmRow];
    __shared__ __attribute__((aligned(16))) int8_t sB[2][kGemmBN][kGemmRow];
    const int per_split = A.ntq * A.ntsv;
    const int sp = (int)blockIdx.x / per_split;
    const int rem = (int)blockIdx.x - sp * per_split;
    const int I = rem / A.ntsv, J = rem - I * A.ntsv;
    // this split's columns [c0, c1), whole steps
    const size_t nsteps = A.stride / kGemmBK;
    const size_t per = (nsteps + A.S - 1) / A.S;
    const size_t c0 = (size_t)sp * per * kGemmBK, c1 = min(A.stride, c0 + per * kGemmBK);
    if (c0 >= c1) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = tid >> 2, lc = (tid & 3) * 16;  // staging: rows lr + 64 j, 16-byte column lc
    // tiled count rows: row r, step column c (a multiple of 64) at
    // (r / 128) 128 stride + 128 c + 64 (r % 128)
    const gptr<const int8_t> ga = glb(A.Q) + (size_t)I * BM * A.stride + lr * 64 + lc;
    const gptr<const int8_t> gb = glb(A.D) + (size_t)J * kGemmBN * A.stride + lr * 64 + lc;
    const size_t s128 = (size_t)128 * A.stride;
    struct SlabA {
        v4i a[BM / 64];
    };
    struct SlabB {
        v4i b[kGemmBN / 64];
    };
    auto gload_a = [&](size_t c, SlabA &x) {
#pragma unroll
        for (int j = 0; j < BM / 64; ++j) x.a[j] = *(gptr<const v4i>)(ga + (size_t)(j >> 1) * s128 + (j & 1) * 4096 + 128 * c);
    };
    auto gload_b = [&](size_t c, SlabB &x) {
#pragma unroll
        for (int j = 0; j < kGemmBN / 64; ++j) x.b[j] = *(gptr<const v4i>)(gb + j * 4096 + 128 * c);
    };
    auto lstore = [&](int buf, const SlabA &xa, const SlabB &xb) {
#pragma unroll
        for (int j = 0; j < BM / 64; ++j) *reinterpret_cast<v4i *>(&sA[buf][lr + 64 * j][lc]) = xa.a[j];
#pragma unroll
        for (int j = 0; j < kGemmBN / 64; ++j) *reinterpret_cast<v4i *>(&sB[buf][lr + 64 * j][lc]) = xb.b[j];
    };
    v16i acc[MT][kGemmNT];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < kGemmNT; ++j) acc[i][j] = v16i{};
    const int fr = lane & 31, fk = 16 * (lane >> 5);
    auto compute = [&](int buf) {
#pragma unroll
        for (int kk = 0; kk < kGemmBK; kk += 32) {
            v4i a[MT], b[kGemmNT];
#pragma unroll
            for (int i = 0; i < MT; ++i) a[i] = *reinterpret_cast<const v4i *>(&sA[buf][wave * WR + 32 * i + fr][kk + fk]);
#pragma unroll
            for (int j = 0; j < kGemmNT; ++j) b[j] = *reinterpret_cast<const v4i *>(&sB[buf][32 * j + fr][kk + fk]);
#pragma unroll
            for (int i = 0; i < MT; ++i)
#pragma unroll
                for (int j = 0; j < kGemmNT; ++j) acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    };
    // Step s: its slabs in LDS buffer s % 2; the query slab of step s + 2
    // (from L2, shared with the split's other blocks) and the resident slab
    // of step s + 3 (streamed from HBM: one more step in flight) are loaded
    // into the register slabs that step s - 1 has stored.  Loads past the
    // split's last step re-read that step (never outside the rows).
    const size_t last = c1 - kGemmBK;
    auto at = [&](int k) { return min(c0 + (size_t)k * kGemmBK, last); };
    SlabA a0, a1;
    SlabB b0, b1, b2, b3;
    gload_a(at(0), a0);
    gload_b(at(0), b0);
    gload_a(at(1), a1);
    gload_b(at(1), b1);
    gload_b(at(2), b2);
    lstore(0, a0, b0);
    __syncthreads();
    auto step = [&](size_t c, int buf, SlabA &lda, const SlabA &sta, SlabB &ldb, const SlabB &stb) {
        gload_b(min(c + 3 * kGemmBK, last), ldb);
        gload_a(min(c + 2 * kGemmBK, last), lda);
        compute(buf);
        lstore(buf ^ 1, sta, stb);
        __syncthreads();
    };
    size_t c = c0;
#pragma unroll 1
    while (true) {
        step(c, 0, a0, a1, b3, b1);
        c += kGemmBK;
        if (c >= c1) break;
        step(c, 1, a1, a0, b0, b2);
        c += kGemmBK;
        if (c >= c1) break;
        step(c, 0, a0, a1, b1, b3);
        c += kGemmBK;
        if (c >= c1) break;
        step(c, 1, a1, a0, b2, b0);
        c += kGemmBK;
        if (c >= c1) break;
    }
    const gptr<uint32_t> C = glb(A.C);
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < kGemmNT; ++j) {
            const int sv = J * kGemmBN + 32 * j + (lane & 31);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int q = I * BM + wave * WR + 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                if (q < A.nq && sv < A.nsv && acc[i][j][v] != 0 && !A.qflag[q])
                    g_atomic_add(C + (size_t)q * A.nsv + sv, (uint32_t)acc[i][j][v]);
            }
        }
}

hipError_t launch_count_rows(const uint64_t *key, const uint32_t *gstart, int nseq, const void *rm, int nset, int w,
                             int8_t *out, size_t stride, uint32_t *flag, hipStream_t st)
{
    if (nseq <= 0 || nset <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((size_t)nseq * (size_t)((nset + kCountRowSets - 1) / kCountRowSets));
    hipLaunchKernelGGL(k_count_rows, dim3(nb), dim3(kThreads), (size_t)4u << w, st, key, gstart, nseq,
                       reinterpret_cast<const ResMask *>(rm), nset, w, out, stride, flag);
    return hipGetLastError();
}

// Query tile of a batch of nq queries: 128 up to 128 queries, else 256.
int rows_gemm_tile_q(int nq) { return nq <= 128 ? 128 : 256; }
int rows_gemm_tile_sv() { return kGemmBN; }

// Column splits of the product: every block runs about as long, so the
// launch takes ceil(blocks / resident) rounds of one split's length; the
// split count minimising rounds / S (the smallest on ties) keeps the last
// round full.
static int gemm_splits(const void *kernel, int tiles, size_t stride)
{
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, 0) != hipSuccess || ncu <= 0 || per_cu <= 0) {
        (void)hipGetLastError();
        return 1;
    }
    const long long resident = (long long)ncu * per_cu;
    const int smax = (int)std::min<size_t>(32, std::max<size_t>(1, stride / kGemmBK));
    int best = 1;
    double best_t = 1e30;
    for (int S = 1; S <= smax; ++S) {
        const double t = (double)(((long long)tiles * S + resident - 1) / resident) / S;
        if (t < best_t - 1e-12) {
            best_t = t;
            best = S;
        }
    }
    return best;
}

hipError_t launch_rows_gemm(const int8_t *Q, const int8_t *D, size_t stride, int nq, int nsv, int S, const uint32_t *qflag,
                            uint32_t *C, hipStream_t st)
{
    if (nq <= 0 || nsv <= 0) return hipSuccess;
    const int bm = rows_gemm_tile_q(nq);
    const int ntq = (nq + bm - 1) / bm, ntsv = (nsv + kGemmBN - 1) / kGemmBN;
    if (S <= 0)
        S = gemm_splits(bm == 128 ? reinterpret_cast<const void *>(&k_rows_gemm<128>) : reinterpret_cast<const void *>(&k_rows_gemm<256>),
                        ntq * ntsv, stride);
    RowsGemmArgs a{Q, D, stride, nq, nsv, ntq, ntsv, S, qflag, C};
    const unsigned nb = (unsigned)((size_t)a.ntq * a.ntsv * S);
    if (bm == 128) hipLaunchKernelGGL(k_rows_gemm<128>, dim3(nb), dim3(kThreads), 0, st, a);
    else hipLaunchKernelGGL(k_rows_gemm<256>, dim3(nb), dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

// K(x,x) from the per-level diagonal counters: Eq. 9 then Eq. 7.  The
// per-level values of up to MM levels stay in registers.
template <int MM>
__global__ __launch_bounds__(kThreads) void k_kdiag_counts(const uint32_t *diag, int n, int M, const int64_t *coef,
                                                           const int64_t *hco, int64_t *Kd)
{
    const int x = blockIdx.x * kThreads + threadIdx.x;
    if (x >= n) return;
    constexpr int UNR = MM <= 16 ? MM : 1;
    int64_t nv[MM];
    int64_t kx = 0;
#pragma unroll UNR
    for (int m = 0; m < MM; ++m) {
        int64_t v = 0;
        if (m <= M) {
            v = diag[(size_t)m * n + x];
#pragma unroll UNR
            for (int j = 0; j < m; ++j) v -= coef[m * (M + 1) + j] * nv[j];
            kx += hco[m] * v;
        }
        nv[m] = v;
    }
    Kd[x] = kx;
}

struct RowsFinArgs {
    const uint32_t *C;
    int32_t nq, nsv, M;
    const int64_t *coef, *hco;
    const int64_t *Kd_sv, *Kd_q;
    const double *alpha;
    double bias;
    double *K_rows;
    int64_t *Nm_rows;
    double *decision;
    double *partial;  // [nq][nchunk] decision sums per SV chunk
    int32_t chunk, nchunk;
    int64_t ldk;      // row stride of K_rows
};

constexpr int kRowsChunk = 512;  // SVs per epilogue block (enough blocks for one query)

// One block per (query, chunk of SVs): Eq. 9 and Eq. 7 per entry, the
// normalisation with K(sv,sv) and K(q,q), and the chunk's part of Eq. 1's
// sum_i alpha_i K-hat(sv_i, q): every thread sums its entries in ascending
// order and the block combines the thread sums in a fixed tree.
template <int MM>
__global__ __launch_bounds__(kThreads) void k_rows_finalize(RowsFinArgs A)
{
    __shared__ double red[kThreads];
    __shared__ int64_t coef[MM * MM], hco[MM];
    const int q = blockIdx.x / A.nchunk, ch = blockIdx.x % A.nchunk, tid = threadIdx.x, M = A.M;
    const int s0 = ch * A.chunk, s1 = min(A.nsv, s0 + A.chunk);
    for (int i = tid; i < (M + 1) * (M + 1); i += kThreads) coef[(i / (M + 1)) * MM + (i % (M + 1))] = A.coef[i];
    for (int i = tid; i <= M; i += kThreads) hco[i] = A.hco[i];
    __syncthreads();
    constexpr int UNR = MM <= 16 ? MM : 1;
    const int64_t kq = A.Kd_q[q];
    double part = 0.0;
    for (int sv = s0 + tid; sv < s1; sv += kThreads) {
        int64_t nv[MM];
        int64_t K = 0;
#pragma unroll UNR
        for (int m = 0; m < MM; ++m) {
            int64_t v = 0;
            if (m <= M) {
                v = A.C[((size_t)m * A.nq + q) * A.nsv + sv];
#pragma unroll UNR
                for (int j = 0; j < m; ++j) v -= coef[m * MM + j] * nv[j];
                K += hco[m] * v;
                if (A.Nm_rows) A.Nm_rows[((size_t)m * A.nq + q) * A.nsv + sv] = v;
            }
            nv[m] = v;
        }
        const int64_t ks = A.Kd_sv[sv];
        const double kh = (kq == 0 || ks == 0) ? 0.0 : (double)K / sqrt((double)ks * (double)kq);
        if (A.K_rows) A.K_rows[(size_t)q * A.ldk + sv] = kh;
        if (A.alpha) part += A.alpha[sv] * kh;
    }
    red[tid] = part;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) A.partial[(size_t)q * A.nchunk + ch] = red[0];
}

// f(q) = b + the chunk sums in ascending chunk order (one thread per query).
__global__ __launch_bounds__(kThreads) void k_rows_decision(RowsFinArgs A)
{
    const int q = blockIdx.x * kThreads + threadIdx.x;
    if (q >= A.nq) return;
    double f = 0.0;
    for (int c = 0; c < A.nchunk; ++c) f += A.partial[(size_t)q * A.nchunk + c];
    A.decision[q] = A.bias + f;
}

size_t res_mask_size() { return sizeof(ResMask); }

void res_mask_fill(void *dst, const MaskDesc &md, int w, int B, int hb, int sb, const uint32_t *boff, const uint32_t *bgrp,
                   const uint32_t *E, const uint4 *gtab)
{
    ResMask r{md, w, B, hb, sb, boff, bgrp, E, gtab};
    *reinterpret_cast<ResMask *>(dst) = r;
}

hipError_t launch_rows(const uint64_t *qkey, const uint32_t *qgstart, int nq, int M, int nsv, int slab, int mchunk,
                       int nitems, const void *rm, const int32_t *lev_first, const int32_t *lev_count, uint32_t *C,
                       unsigned long long *updates, int dense_level, const uint32_t *qflag, hipStream_t st)
{
    if (nq <= 0) return hipSuccess;
    RowsArgs a{qkey, qgstart, nq, M, nsv, slab, (nsv + slab - 1) / slab, mchunk, reinterpret_cast<const ResMask *>(rm),
               lev_first, lev_count, C, updates, dense_level, qflag};
    const unsigned nb = (unsigned)((size_t)nq * nitems * a.nslab);
    hipLaunchKernelGGL(k_rows_accumulate, dim3(nb), dim3(kThreads), (size_t)slab * 4, st, a);
    return hipGetLastError();
}

hipError_t launch_kdiag_counts(const uint32_t *diag, int n, int M, const int64_t *coef, const int64_t *hco, int64_t *Kd,
                               hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const dim3 grid((n + kThreads - 1) / kThreads);
    if (M < 8) hipLaunchKernelGGL(k_kdiag_counts<8>, grid, dim3(kThreads), 0, st, diag, n, M, coef, hco, Kd);
    else if (M < 16) hipLaunchKernelGGL(k_kdiag_counts<16>, grid, dim3(kThreads), 0, st, diag, n, M, coef, hco, Kd);
    else hipLaunchKernelGGL(k_kdiag_counts<65>, grid, dim3(kThreads), 0, st, diag, n, M, coef, hco, Kd);
    return hipGetLastError();
}

size_t rows_partial_count(int nq, int nsv) { return (size_t)nq * (size_t)((nsv + kRowsChunk - 1) / kRowsChunk); }

hipError_t launch_rows_finalize(const uint32_t *C, int nq, int nsv, int M, const int64_t *coef, const int64_t *hco,
                                const int64_t *Kd_sv, const int64_t *Kd_q, const double *alpha, double bias, double *K_rows,
                                int64_t ldk, int64_t *Nm_rows, double *decision, double *partial, hipStream_t st)
{
    if (nq <= 0) return hipSuccess;
    const int nchunk = (nsv + kRowsChunk - 1) / kRowsChunk;
    RowsFinArgs a{C, nq, nsv, M, coef, hco, Kd_sv, Kd_q, alpha, bias, K_rows, Nm_rows, decision, partial, kRowsChunk, nchunk,
                  ldk > 0 ? ldk : (int64_t)nsv};
    const dim3 grid((unsigned)(nq * nchunk));
    if (M < 8) hipLaunchKernelGGL(k_rows_finalize<8>, grid, dim3(kThreads), 0, st, a);
    else if (M < 16) hipLaunchKernelGGL(k_rows_finalize<16>, grid, dim3(kThreads), 0, st, a);
    else hipLaunchKernelGGL(k_rows_finalize<65>, grid, dim3(kThreads), 0, st, a);
    if (decision) hipLaunchKernelGGL(k_rows_decision, dim3((nq + kThreads - 1) / kThreads), dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

// out[r][c0 + c] = out[c0 + c][r] for r < rows, c < cols (row stride ld):
// the block above the diagonal from the block below it, through 32 x 32 LDS
// tiles.
__global__ __launch_bounds__(kThreads) void k_mirror_block(double *out, int64_t ld, int rows, int c0, int cols)
{
    __shared__ double tile[32][33];
    const int tr = blockIdx.y * 32, tc = blockIdx.x * 32;  // tile origin in (row r, column c)
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
    for (int k = ty; k < 32; k += 8) {
        const int c = tc + k, r = tr + tx;  // read out[c0 + c][r], coalesced along r
        if (c < cols && r < rows) tile[k][tx] = out[(size_t)(c0 + c) * ld + r];
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int r = tr + k, c = tc + tx;  // write out[r][c0 + c], coalesced along c
        if (r < rows && c < cols) out[(size_t)r * ld + c0 + c] = tile[tx][k];
    }
}

hipError_t launch_mirror_block(double *out, int64_t ld, int rows, int c0, int cols, hipStream_t st)
{
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
    hipLaunchKernelGGL(k_mirror_block, grid, dim3(kThreads), 0, st, out, ld, rows, c0, cols);
    return hipGetLastError();
}

hipError_t init_rows_attributes(size_t lds)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rows_accumulate), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds);
}

}  // namespace gk
