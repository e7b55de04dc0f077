// gfx950 kernels of the plain Gram path: validation, g-mer extraction,
// hash-bucket partition (count / scan / scatter), per-bucket LDS radix sort
// with group segmentation, row-owned accumulation of the cumulative mismatch
// profiles, and the inclusion-exclusion / kernel / normalisation epilogue.
#include <type_traits>

#include "common.h"
#include "launch.h"

namespace gk {

// ---------------------------------------------------------------- fills --
__global__ void k_fill_u64(uint64_t *p, size_t n, uint64_t v)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u32(uint32_t *p, size_t n, uint32_t v)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ------------------------------------------------------------ validation --
// Every symbol code must lie in [0, sigma); a violation sets bit 0 of err.
__global__ __launch_bounds__(kThreads) void k_validate(const JobDev *__restrict__ jobs, const uint32_t *__restrict__ bprefix, int njobs)
{
    const int j = find_item(bprefix, njobs, blockIdx.x);
    const JobDev &J = jobs[j];
    const int64_t i0 = (int64_t)(blockIdx.x - bprefix[j]) * (kThreads * 16);
    bool bad = false;
    for (int q = 0; q < 16; ++q) {
        const int64_t i = i0 + q * kThreads + threadIdx.x;
        if (i < J.nsym) bad |= ((uint8_t)J.seqs[i] >= (uint32_t)J.sigma);
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(J.err, 1);
}

// ------------------------------------------------------------- extraction --
// g-mer t of sequence X at position p: key = sum_j x[p+j] << (b*(g-1-j))
// (Section 2.2, step 1).  One thread per g-mer.
__global__ __launch_bounds__(kThreads) void k_extract(const JobDev *__restrict__ jobs, const uint32_t *__restrict__ bprefix, int njobs)
{
    const int j = find_item(bprefix, njobs, blockIdx.x);
    const JobDev &J = jobs[j];
    const uint32_t t = (blockIdx.x - bprefix[j]) * kThreads + threadIdx.x;
    if (t >= J.T) return;
    const int X = (int)last_le(J.gstart, (uint32_t)J.N + 1u, t);
    const uint32_t p = t - J.gstart[X];
    const int8_t *s = J.seqs + J.seq_off[X] + p;
    const uint64_t fm = (1ull << J.b) - 1ull;
    uint64_t key = 0;
    for (int q = 0; q < J.g; ++q) key = (key << J.b) | ((uint64_t)(uint8_t)s[q] & fm);
    J.key[t] = J.kshift ? key | ((uint64_t)X << J.kshift) : key;
    J.sid[t] = (uint32_t)X;
}

// --------------------------------------------------------- bucket count --
// Histogram of bucket = top B bits of mix_w(reduced key) per mask, over
// tiles of kCountTile g-mers (larger than the scatter's: fewer global adds).
__global__ __launch_bounds__(kCountThreads) void k_bucket_count(const MaskWork *__restrict__ items, const uint32_t *__restrict__ bprefix,
                                                                int nitems, uint32_t uniform)
{
    extern __shared__ uint32_t hist[];
    int it;
    uint32_t tile;
    map_block(bprefix, nitems, uniform, blockIdx.x, it, tile);
    const MaskWork &W = items[it];
    const uint32_t t0 = tile * kCountTile;
    if (t0 >= W.T) return;
    const uint32_t nb = 1u << W.B;
    for (uint32_t i = threadIdx.x; i < nb; i += kCountThreads) hist[i] = 0;
    __syncthreads();
    constexpr int Q = 8;  // keys in flight per thread
#pragma unroll 1
    for (int h = 0; h < kCountTile / kCountThreads; h += Q) {
        uint64_t key[Q], rk[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {  // every load issued before any is used
            const uint32_t t = t0 + (h + q) * kCountThreads + threadIdx.x;
            key[q] = t < W.T ? glb(W.key)[t] : 0ull;
        }
        compact_keys<Q>(key, rk, W.md);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const uint32_t t = t0 + (h + q) * kCountThreads + threadIdx.x;
            if (t < W.T) atomicAdd(&hist[(uint32_t)(mix_w(rk[q], W.w) >> W.hb)], 1u);
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nb; i += kCountThreads)
        if (hist[i]) g_atomic_add(glb(W.bcnt) + i, hist[i]);
}

// ------------------------------------------------------- bucket scatter --
// Place (composite, g-mer index) of every g-mer into its bucket: composites
// of at most 32 bits as one packed word composite << 32 | index, wider ones
// in the composite array with the index beside it.  The order inside a
// bucket is arbitrary; the bucket sort restores it.
__global__ __launch_bounds__(kScatterThreads) void k_bucket_scatter(const MaskWork *__restrict__ items, const uint32_t *__restrict__ bprefix,
                                                             int nitems, uint32_t uniform)
{
    extern __shared__ uint32_t hist[];
    int it;
    uint32_t tile;
    map_block(bprefix, nitems, uniform, xcd_order(blockIdx.x, gridDim.x), it, tile);
    const MaskWork &W = items[it];
    const uint32_t t0 = tile * kTile;
    if (t0 >= W.T) return;
    const uint32_t nb = 1u << W.B;
    constexpr int Q = kTile / kScatterThreads;
    for (uint32_t i = threadIdx.x; i < nb; i += kScatterThreads) hist[i] = 0;
    __syncthreads();
    uint32_t bk[Q], rk[Q];
    uint64_t cp[Q], kv[Q];
    const uint64_t hmask = bits_mask(W.hb);
#pragma unroll
    for (int q = 0; q < Q; ++q) {  // every load issued before any is used
        const uint32_t t = t0 + q * kScatterThreads + threadIdx.x;
        kv[q] = t < W.T ? glb(W.key)[t] : 0ull;
    }
    compact_keys<Q>(kv, cp, W.md);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const uint32_t t = t0 + q * kScatterThreads + threadIdx.x;
        bk[q] = 0xFFFFFFFFu;
        if (t < W.T) {
            const uint64_t h = mix_w(cp[q], W.w);
            bk[q] = (uint32_t)(h >> W.hb);
            cp[q] = ((h & hmask) << W.sb) | (W.kshift ? (kv[q] >> W.kshift) : (uint64_t)glb(W.sid)[t]);
            rk[q] = atomicAdd(&hist[bk[q]], 1u);
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nb; i += kScatterThreads) {
        const uint32_t c = hist[i];
        if (c) hist[i] = g_atomic_add(glb(W.bcur) + i, c);
    }
    __syncthreads();
    const bool narrow = W.cb + W.ib <= 64;
    if (W.i4) {  // the sort stores only nonzero 4-byte records: clear the tile's
        const gptr<uint32_t> info4 = (gptr<uint32_t>)glb(W.info);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const uint32_t t = t0 + q * kScatterThreads + threadIdx.x;
            if (t < W.T) info4[t] = 0u;
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (bk[q] != 0xFFFFFFFFu) {
            const uint32_t pos = hist[bk[q]] + rk[q];
            const uint32_t t = t0 + q * kScatterThreads + threadIdx.x;
            if (narrow) {
                glb(W.comp)[pos] = (cp[q] << W.ib) | t;
            } else {
                glb(W.comp)[pos] = cp[q];
                glb(W.idx)[pos] = t;
            }
        }
    }
}

// ---------------------------------------------------------- accumulation --
// One block owns row X of C_m for one level m, as int32 counters in LDS.  For
// each mask of the level and each g-mer of X that leads a run (X's entry in
// its group), the entries from X's own to the group end -- exactly the
// sequences Y >= X of the group, since entries are sequence-sorted -- add
// count_X * count_Y to row[Y] (Algorithm 1 countAndUpdate, upper triangle).
// X's own entry is count_X^2 on the diagonal, summed in registers; a run with
// one more entry carries it in its info; longer tails are read from the run
// entries.  Each wave consumes its own chunks of 128 (mask, g-mer) items, two
// per lane, whose records were loaded during the previous chunk; the chunk's
// tails are laid end to end (a wave scan of their lengths) and the lanes walk
// that sequence kAccWindow updates at a time (eight gathers in flight per
// lane): one bit per tail start in LDS, read back as 64-bit words, and a
// popcount below the lane give each update its tail without a search.  The
// loop has no block barrier.  The row is then added into the int64 C_m.
// When a row does not fit the LDS, each block takes a slab of its columns
// [y0, y1) and cuts every tail to the entries of those sequences (a search
// of the sequence-sorted entries); slabs below the diagonal have no work.
constexpr int kAccWindow = 512;
constexpr int kAccU = kAccWindow / 64;
constexpr int kAccItems = 2;  // items per lane in one wave chunk

// First index in [lo, hi) whose entry's sequence is >= s (hi if none); the
// entries of one group are sorted by sequence.
template <typename Ent>
__device__ __forceinline__ uint32_t first_seq_at_least(const Ent *E, uint32_t lo, uint32_t hi, uint32_t s, uint32_t sidmask)
{
    const gptr<const Ent> e = glb(E);
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((e[mid] & sidmask) < s) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}
constexpr int kAccTails = 64 * kAccItems;  // tails per wave chunk at most
struct AccLds {
    uint64_t tbase[kWaves][kAccTails];  // per tail: entry address - 4 * its start in the sequence
    uint32_t tcx[kWaves][kAccTails];    // per tail: count_X
    uint32_t mark[kWaves][kAccWindow / 32];  // tail starts in the current window, one bit each
};

// The block's work with 4-byte records (I4) or uint2 records.
template <bool I4>
__device__ __forceinline__ void accumulate_row(const JobDev *__restrict__ jobs, const MaskWork *__restrict__ items,
                                               const AccWork &A, int flat, uint32_t *acc, AccLds &L,
                                               unsigned long long *updates)
{
    auto &tbase = L.tbase;
    auto &tcx = L.tcx;
    auto &mark = L.mark;
    const JobDev &J = jobs[A.job];
    const int X = flat / A.nslab;
    const int N = J.N;
    // this block's columns [y0, y1) of row X; it writes [max(X, y0), y1)
    const int y0 = (flat - X * A.nslab) * A.slab, y1 = min(N, y0 + A.slab);
    if (y1 <= X) return;  // the slab lies below the diagonal
    const bool whole = A.nslab == 1;
    const int ylo = max(X, y0);
    const bool own_col = X >= y0;  // the diagonal entry is in this slab
    const int tid = threadIdx.x, lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
    const int sb = J.sb;
    const uint32_t sidmask = (uint32_t)bits_mask(sb);
    const uint32_t lmask = (uint32_t)bits_mask(sb + 1);
    const uint32_t t0 = J.gstart[X];
    const uint32_t ng = J.gstart[X + 1] - t0;
    const gptr<int64_t> crow = glb(J.C) + ((size_t)A.level * N + X) * (size_t)N;
    if (ng == 0 || A.nmask == 0) {  // nothing to add: a stored row is 0
        if (A.first)
            for (int Y = ylo + tid; Y < y1; Y += kThreads) crow[Y] = 0;
        return;
    }
    // the first mask's arrays; mask s's are mstride * s bytes further
    const MaskWork &W0 = items[A.mfirst];
    const uint64_t info0 = reinterpret_cast<uint64_t>(W0.info), ent0 = reinterpret_cast<uint64_t>(W0.E);
    const uint32_t T = W0.T;
    const int64_t mstride = A.mstride;
    // 4-byte records leave the diagonal's unit terms to a base of one per
    // g-mer and mask
    using Rec = std::conditional_t<I4, uint32_t, uint64_t>;
    // and 16-bit run entries (count field 0: the count is in the escape
    // slot T entries further)
    using Ent = std::conditional_t<I4, uint16_t, uint32_t>;
    constexpr uint32_t ES = sizeof(Ent);
    if (lane < kAccWindow / 32) mark[wid][lane] = 0;
    uint32_t nupd = 0;           // this lane's diagonal and inline pair updates
    unsigned long long wupd = 0;  // the wave's gathered pair updates (profiling count)
    uint32_t *const accy = acc - y0;  // column Y at accy[Y]
    // The masks are taken mstep at a time, the int32 row flushed into the
    // int64 C_m after each step: one mask adds at most ng_X * ng_Y to an
    // entry, and the planner picks mstep so that mstep * maxng^2 < 2^32.
    const int mstep = A.mstep > 0 ? min(A.mstep, A.nmask) : A.nmask;
#pragma unroll 1
    for (int ms0 = 0; ms0 < A.nmask; ms0 += mstep) {
    const int nmk = min(mstep, A.nmask - ms0);
    for (int i = tid; i < A.Npad; i += kThreads) acc[i] = 0;
    __syncthreads();
    if (I4 && own_col && tid == 0) {  // every g-mer of X leads or joins one run per mask: 1 each
        atomicAdd(&acc[X - y0], (uint32_t)nmk * ng);
        nupd += (uint32_t)nmk * ng;
    }
    uint32_t dsum = 0;  // this lane's diagonal terms
    // item q = (mask ms0 + q / ng, g-mer t0 + q % ng): its mask's byte offset
    // and its record; the next chunk's records are loaded while this
    // chunk's tails are walked
    const uint32_t total = (uint32_t)nmk * ng;
    auto item_mask = [&](uint32_t q, uint32_t &t) -> int64_t {
        const uint32_t s = q / ng;
        t = t0 + (q - s * ng);
        return (int64_t)(ms0 + (int)s) * mstride;
    };
    auto load_rec = [&](uint32_t q) -> Rec {
        if (q >= total) return 0;
        uint32_t t;
        const int64_t mo = item_mask(q, t);
        return *(gptr<const Rec>)(const Rec *)(info0 + (uint64_t)mo + sizeof(Rec) * (uint64_t)t);
    };
    // One item: its diagonal term and inline pair go to the row at once;
    // a longer tail is returned as (length, address of its first entry).
    auto item = [&](uint32_t q, Rec rec, uint32_t &len, uint64_t &ebase, uint32_t &cx) {
        len = 0;
        ebase = 0;
        cx = 0;
        if (q >= total) return;
        uint32_t t;
        const int64_t mo = item_mask(q, t);
        const uint64_t ents = ent0 + (uint64_t)mo;  // this mask's run entries
        // the run X has in this group: entries from its own to the group
        // end (tail), its count, and either the group's last entry inline
        // or its own entry index
        uint32_t tail, xi = 0;
        uint32_t dterm = 0;  // X's diagonal term from this item, beyond the base
        bool inl2 = false;
        if constexpr (I4) {
            const uint32_t v = rec;
            tail = v & 127u;
            const uint32_t pay = v >> 11;
            if (tail == 0) {
                dterm = 0u - (v >> 8);  // count-matrix run: count^2 comes from the product
            } else if (tail == 1) {
                cx = pay;
            } else if (v & 128u) {
                cx = (v >> 8) & 7u;
                inl2 = true;
                xi = pay;
            } else {
                xi = pay;
                if (tail == 127u) tail = *(gptr<const uint32_t>)(info0 + (uint64_t)mo + 4ull * ((uint64_t)T + xi));
                cx = (v >> 8) & 7u;
                if (!cx) {
                    cx = (uint32_t)*(gptr<const uint16_t>)(ents + 2ull * xi) >> sb;
                    if (!cx) cx = *(gptr<const uint16_t>)(ents + 2ull * ((uint64_t)T + xi));
                }
            }
            if (tail) dterm = cx * cx - cx;
        } else {
            const uint32_t y = (uint32_t)(rec >> 32);
            tail = y & lmask;
            cx = y >> (sb + 1);
            xi = (uint32_t)rec;
            inl2 = tail == 2;
            if (tail) dterm = cx * cx;
        }
        if (own_col && dterm) {
            dsum += dterm;
            if (!I4) ++nupd;
        }
        if (inl2) {
            const uint32_t ys = xi & sidmask;
            if (whole || (ys >= (uint32_t)y0 && ys < (uint32_t)y1)) {
                atomicAdd(&accy[ys], cx * (xi >> sb));
                ++nupd;
            }
        } else if (tail >= 2) {
            // entries [e0, e1): sequences above X in ascending order
            const Ent *E = reinterpret_cast<const Ent *>(ents);
            uint32_t e0 = xi + 1, e1 = xi + tail;
            if (!whole) {
                if (y0 > X + 1) e0 = first_seq_at_least(E, e0, e1, (uint32_t)y0, sidmask);
                if (y1 < N) e1 = first_seq_at_least(E, e0, e1, (uint32_t)y1, sidmask);
            }
            len = e1 - e0;
            ebase = ents + ES * (uint64_t)e0;
        }
    };
    constexpr uint32_t kStep = kThreads * kAccItems;  // items per block round
    Rec rnext[kAccItems];
#pragma unroll
    for (int i = 0; i < kAccItems; ++i) rnext[i] = load_rec((uint32_t)(wid * kAccTails + i * 64 + lane));
    for (uint32_t c0 = (uint32_t)wid * kAccTails; c0 < total; c0 += kStep) {
        uint32_t len[kAccItems], cxv[kAccItems];
        uint64_t eb[kAccItems];
        uint32_t lsum = 0;
#pragma unroll
        for (int i = 0; i < kAccItems; ++i) {
            const uint32_t q = c0 + (uint32_t)(i * 64 + lane);
            const Rec rec = rnext[i];
            rnext[i] = load_rec(q + kStep);
            item(q, rec, len[i], eb[i], cxv[i]);
            lsum += len[i];
        }
        // the chunk's tails laid end to end in (lane, item) order
        const uint32_t inc = wave_incl_scan(lsum);
        const uint32_t work = __builtin_amdgcn_readlane(inc, 63);
        if (work == 0) continue;  // wave-uniform
        wupd += work;
        uint32_t start[kAccItems];
        {
            uint32_t kk = 0;  // nonempty tails of the lanes below
#pragma unroll
            for (int i = 0; i < kAccItems; ++i) kk += lanes_below(__ballot(len[i] > 0));
            uint32_t s = inc - lsum;
#pragma unroll
            for (int i = 0; i < kAccItems; ++i) {
                start[i] = s;
                s += len[i];
                if (len[i] > 0) {
                    tbase[wid][kk] = eb[i] - ES * (uint64_t)start[i];
                    tcx[wid][kk] = cxv[i];
                    ++kk;
                }
            }
        }
        uint32_t done = 0;  // tails started before the window
#pragma unroll 1
        for (uint32_t w = 0; w < work; w += kAccWindow) {
#pragma unroll
            for (int i = 0; i < kAccItems; ++i)
                if (len[i] > 0 && start[i] >= w && start[i] < w + kAccWindow)
                    atomicOr(&mark[wid][(start[i] - w) >> 5], 1u << ((start[i] - w) & 31u));
            wave_sync();
            uint64_t st[kAccU];
#pragma unroll
            for (int u = 0; u < kAccU; ++u) st[u] = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)mark[wid][2 * u + 1]) << 32) |
                        (uint32_t)__builtin_amdgcn_readfirstlane((int)mark[wid][2 * u]);  // wave-uniform
            wave_sync();
            if (lane < kAccWindow / 32) mark[wid][lane] = 0;
            // sub-steps past the work are skipped (uniform conditions)
            {
                uint32_t k[kAccU], ent[kAccU];
#pragma unroll
                for (int u = 0; u < kAccU; ++u) {
                    if (w + 64u * u < work) {
                        k[u] = done + lanes_below(st[u]) + (uint32_t)((st[u] >> lane) & 1ull) - 1u;
                        done += (uint32_t)__popcll(st[u]);
                    }
                }
#pragma unroll
                for (int u = 0; u < kAccU; ++u) {
                    if (w + 64u * u < work) {
                        const uint32_t p = min(w + 64u * u + (uint32_t)lane, work - 1u);
                        ent[u] = *(gptr<const Ent>)(const Ent *)(tbase[wid][k[u]] + ES * (uint64_t)p);
                    }
                }
#pragma unroll
                for (int u = 0; u < kAccU; ++u) {
                    if (w + 64u * u < work) {
                        // counts stay below 2^16 (g-mers per sequence): 24-bit products
                        const uint32_t p = w + 64u * u + (uint32_t)lane;
                        if (p < work) {
                            uint32_t cy = ent[u] >> sb;
                            if (I4 && cy == 0)  // escaped count
                                cy = *(gptr<const uint16_t>)(const uint16_t *)(tbase[wid][k[u]] + 2ull * ((uint64_t)T + p));
                            atomicAdd(&accy[ent[u] & sidmask], __umul24(tcx[wid][k[u]], cy));
                        }
                    }
                }
            }
        }
        wave_sync();
    }
    {
        const uint32_t d = wave_incl_scan(dsum);  // nonzero only when X is in the slab
        if (lane == 63 && d) atomicAdd(&acc[X - y0], d);
    }
    __syncthreads();
    const bool store = A.first && ms0 == 0;
    if (store) {
        for (int Y = ylo + tid; Y < y1; Y += kThreads) crow[Y] = (int64_t)acc[Y - y0];
    } else {
        for (int Y = ylo + tid; Y < y1; Y += kThreads) {
            const uint32_t v = acc[Y - y0];
            if (v) crow[Y] += (int64_t)v;
        }
    }
    __syncthreads();  // the row is read before the next step clears it
    }
    if (updates) {  // profiling count, spread over 256 slots by block
        const uint32_t u = wave_incl_scan(nupd);
        if (lane == 63) atomicAdd(updates + (blockIdx.x & 255u), wupd + (unsigned long long)u);
    }
}

__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_accumulate(
    const JobDev *__restrict__ jobs, const MaskWork *__restrict__ items, const AccWork *__restrict__ aw,
    const uint32_t *__restrict__ bprefix, int nacc, unsigned long long *updates)
{
    extern __shared__ uint32_t acc[];
    __shared__ AccLds L;
    const int a = find_item(bprefix, nacc, blockIdx.x);
    const AccWork &A = aw[a];
    const int flat = (int)(blockIdx.x - bprefix[a]);
    // the record format is the job's (uniform over its masks)
    if (A.nmask > 0 && items[A.mfirst].i4) accumulate_row<true>(jobs, items, A, flat, acc, L, updates);
    else accumulate_row<false>(jobs, items, A, flat, acc, L, updates);
}

// -------------------------------------------------------------- epilogue --
// K_XX from the diagonal of C: Eq. 9 then Eq. 7.
template <int MM>
__global__ __launch_bounds__(kThreads) void k_diag(const JobDev *__restrict__ jobs, const uint32_t *__restrict__ bprefix, int njobs)
{
    const int j = find_item(bprefix, njobs, blockIdx.x);
    const JobDev &J = jobs[j];
    const int X = (int)((blockIdx.x - bprefix[j]) * kThreads + threadIdx.x);
    if (X >= J.N) return;
    const int M = J.M, N = J.N;
    int64_t nv[MM];
    int64_t kx = 0;
    for (int m = 0; m <= M; ++m) {
        int64_t v = J.C[((size_t)m * N + X) * N + X];
        if (J.dref && J.dref[m].P) v += dense_part(J.dref[m], dense_splits_used(J.dref[m]), X, X);
        for (int jj = 0; jj < m; ++jj) v -= J.coef[m * (M + 1) + jj] * nv[jj];
        nv[m] = v;
        kx += J.hco[m] * v;
    }
    J.Kd[X] = kx;
}

// One block per 32x32 tile (I <= J) of the upper triangle: inclusion-
// exclusion (Eq. 9), K (Eq. 7) and the cosine normalisation for every entry
// x <= y, written to (x, y) and, through an LDS transpose, to (y, x).  QN
// entries per thread (1024 / QN threads), so that the per-level values of
// up to MM levels stay in registers.
// Tile (I, J), I <= J, of the f-th upper tile in row-major order of an
// nt x nt tile grid: row I starts at S(I) = I nt - I (I - 1) / 2.
__device__ __forceinline__ void upper_tile(int f, int nt, int &I, int &J)
{
    const double b = 2.0 * nt + 1.0;
    int i = (int)((b - sqrt(b * b - 8.0 * f)) * 0.5);
    i = max(0, min(i, nt - 1));
    auto S = [nt](int r) { return r * nt - r * (r - 1) / 2; };
    while (i + 1 < nt && S(i + 1) <= f) ++i;
    while (i > 0 && S(i) > f) --i;
    I = i;
    J = i + (f - S(i));
}

template <int MM, int QN>
__global__ __launch_bounds__(1024 / QN) void k_finalize(const JobDev *__restrict__ jobs, const uint32_t *__restrict__ bprefix, int njobs)
{
    constexpr int FT = 1024 / QN, RS = FT / 32;  // threads; rows apart of a thread's entries
    __shared__ int64_t coef[MM * MM];
    __shared__ int64_t hco[MM];
    __shared__ int64_t tile[32][33];
    __shared__ int nsplit[MM];
    __shared__ DenseRef dref[MM];
    const int j = find_item(bprefix, njobs, blockIdx.x);
    const JobDev &Jb = jobs[j];
    const int N = Jb.N, M = Jb.M;
    const int nt = (N + 31) / 32;
    const int flat = (int)(blockIdx.x - bprefix[j]);
    int I, Jt;
    upper_tile(flat, nt, I, Jt);
    const int tid = threadIdx.x;
    for (int i = tid; i < (M + 1) * (M + 1); i += FT) coef[(i / (M + 1)) * MM + (i % (M + 1))] = Jb.coef[i];
    for (int i = tid; i <= M; i += FT) {
        hco[i] = Jb.hco[i];
        nsplit[i] = (Jb.dref && Jb.dref[i].P) ? dense_splits_used(Jb.dref[i]) : 0;
        if (nsplit[i]) dref[i] = Jb.dref[i];
    }
    __syncthreads();
    const int c = tid & 31;
    // level loops are unrolled over the compile-time bound so the per-level
    // values stay in registers
    constexpr int UNR = MM <= 16 ? MM : 1;
    int64_t nv[QN][MM];
    int64_t kv[QN];
    bool valid[QN];
#pragma unroll
    for (int q = 0; q < QN; ++q) {
        const int r = (tid >> 5) + RS * q;
        const int x = I * 32 + r, y = Jt * 32 + c;
        valid[q] = (x < N) && (y < N) && (I < Jt || r <= c);
        kv[q] = 0;
        if (valid[q]) {
#pragma unroll UNR
            for (int m = 0; m < MM; ++m) {
                int64_t v = 0;
                if (m <= M) {
                    v = glb(Jb.C)[((size_t)m * N + x) * N + y];
                    if (nsplit[m]) v += dense_part(dref[m], nsplit[m], x, y);
#pragma unroll UNR
                    for (int jj = 0; jj < m; ++jj) v -= coef[m * MM + jj] * nv[q][jj];
                    kv[q] += hco[m] * v;
                }
                nv[q][m] = v;
            }
        }
    }
    __syncthreads();  // every read of C precedes any write (C may alias Nm_out)
    auto emit = [&](gptr<int64_t> out, auto value_of) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            const int r = (tid >> 5) + RS * q;
            if (valid[q]) {
                const int64_t v = value_of(q);
                __builtin_nontemporal_store(v, &out[(size_t)(I * 32 + r) * N + (Jt * 32 + c)]);
                tile[r][c] = v;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            const int r = (tid >> 5) + RS * q;
            const int sx = I * 32 + c, sy = Jt * 32 + r;  // source element (sx, sy), sx <= sy
            if (sx < N && sy < N && (I < Jt || c <= r)) __builtin_nontemporal_store(tile[c][r], &out[(size_t)sy * N + sx]);
        }
        __syncthreads();
    };
    if (Jb.Nm_out) {
#pragma unroll UNR
        for (int m = 0; m < MM; ++m) {
            if (m > M) continue;
            emit(glb(Jb.Nm_out) + (size_t)m * N * N, [&](int q) __attribute__((always_inline)) { return nv[q][m]; });
        }
    }
    if (Jb.Cm_out) {
#pragma unroll UNR
        for (int m = 0; m < MM; ++m) {
            if (m > M) continue;
            emit(glb(Jb.Cm_out) + (size_t)m * N * N, [&](int q) __attribute__((always_inline)) {
                int64_t v = nv[q][m];
#pragma unroll UNR
                for (int jj = 0; jj < m; ++jj) v += coef[m * MM + jj] * nv[q][jj];
                return v;
            });
        }
    }
    if (Jb.K_out) {
        const gptr<int64_t> kout = glb(reinterpret_cast<int64_t *>(Jb.K_out));
        emit(kout, [&](int q) {
            const int r = (tid >> 5) + RS * q;
            const int64_t kx = glb(Jb.Kd)[I * 32 + r], ky = glb(Jb.Kd)[Jt * 32 + c];
            const double kh = (kx == 0 || ky == 0) ? 0.0 : (double)kv[q] / sqrt((double)kx * (double)ky);
            return __double_as_longlong(kh);
        });
    }
}

// --------------------------------------------------------------- launchers --
static inline unsigned nblk(size_t n, unsigned per) { return (unsigned)((n + per - 1) / per); }

hipError_t launch_fill_u64(uint64_t *p, size_t n, uint64_t v, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    unsigned g = nblk(n, kThreads);
    if (g > 65536u) g = 65536u;
    hipLaunchKernelGGL(k_fill_u64, dim3(g), dim3(kThreads), 0, st, p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    unsigned g = nblk(n, kThreads);
    if (g > 65536u) g = 65536u;
    hipLaunchKernelGGL(k_fill_u32, dim3(g), dim3(kThreads), 0, st, p, n, v);
    return hipGetLastError();
}
hipError_t launch_validate(const JobDev *jobs, const uint32_t *bprefix, int njobs, uint32_t nblocks, hipStream_t st)
{
    if (!nblocks) return hipSuccess;
    hipLaunchKernelGGL(k_validate, dim3(nblocks), dim3(kThreads), 0, st, jobs, bprefix, njobs);
    return hipGetLastError();
}
hipError_t launch_extract(const JobDev *jobs, const uint32_t *bprefix, int njobs, uint32_t nblocks, hipStream_t st)
{
    if (!nblocks) return hipSuccess;
    hipLaunchKernelGGL(k_extract, dim3(nblocks), dim3(kThreads), 0, st, jobs, bprefix, njobs);
    return hipGetLastError();
}
hipError_t launch_bucket_count(const MaskWork *items, const uint32_t *bprefix, int nitems, uint32_t uniform, uint32_t nblocks,
                               int maxB, hipStream_t st)
{
    if (!nblocks) return hipSuccess;
    hipLaunchKernelGGL(k_bucket_count, dim3(nblocks), dim3(kCountThreads), (size_t)4u << maxB, st, items, bprefix, nitems, uniform);
    return hipGetLastError();
}
hipError_t launch_bucket_scatter(const MaskWork *items, const uint32_t *bprefix, int nitems, uint32_t uniform, uint32_t nblocks,
                                 int maxB, hipStream_t st)
{
    if (!nblocks) return hipSuccess;
    hipLaunchKernelGGL(k_bucket_scatter, dim3(nblocks), dim3(kScatterThreads), (size_t)4u << maxB, st, items, bprefix, nitems, uniform);
    return hipGetLastError();
}
hipError_t launch_accumulate(const JobDev *jobs, const MaskWork *items, const AccWork *aw, const uint32_t *bprefix, int nacc,
                             uint32_t nblocks, size_t lds_bytes, unsigned long long *updates, hipStream_t st)
{
    if (!nblocks) return hipSuccess;
    hipLaunchKernelGGL(k_accumulate, dim3(nblocks), dim3(kThreads), lds_bytes, st, jobs, items, aw, bprefix, nacc, updates);
    return hipGetLastError();
}

// Reference rate for the row accumulation: every thread adds 1 to row
// counters at pseudo-random LDS addresses (a 32-bit LCG, Numerical Recipes
// constants), iters times.  The row is summed afterwards so that the adds
// are kept; the sum equals threads * iters and is stored only if it is not.
__global__ __launch_bounds__(kThreads) void k_lds_atomic_probe(int row_words, int iters, uint32_t *sink)
{
    extern __shared__ uint32_t row[];
    for (int i = threadIdx.x; i < row_words; i += kThreads) row[i] = 0;
    __syncthreads();
    uint32_t x = blockIdx.x * kThreads + threadIdx.x + 1u;
    const uint32_t msk = (uint32_t)row_words - 1u;
    for (int it = 0; it < iters; ++it) {
        x = x * 1664525u + 1013904223u;
        atomicAdd(&row[(x >> 12) & msk], 1u);
    }
    __syncthreads();
    uint32_t sum = 0;
    for (int i = threadIdx.x; i < row_words; i += kThreads) sum += row[i];
    __shared__ uint32_t tot;
    if (threadIdx.x == 0) tot = 0;
    __syncthreads();
    atomicAdd(&tot, sum);
    __syncthreads();
    if (threadIdx.x == 0 && tot != (uint32_t)(kThreads * iters)) sink[0] = tot;
}

hipError_t probe_lds_atomics(int row_words, double *updates_per_s)
{
    constexpr int kBlocks = 2048, kIters = 4096;
    uint32_t *sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t err = hipMalloc(&sink, sizeof(uint32_t));
    if (err == hipSuccess) err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    float ms = 0.f;
    if (err == hipSuccess) {
        const size_t lds = (size_t)row_words * 4;
        hipLaunchKernelGGL(k_lds_atomic_probe, dim3(kBlocks), dim3(kThreads), lds, nullptr, row_words, kIters, sink);
        (void)hipEventRecord(e0, nullptr);
        hipLaunchKernelGGL(k_lds_atomic_probe, dim3(kBlocks), dim3(kThreads), lds, nullptr, row_words, kIters, sink);
        (void)hipEventRecord(e1, nullptr);
        err = hipGetLastError();
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (sink) (void)hipFree(sink);
    if (err == hipSuccess) *updates_per_s = (double)kBlocks * kThreads * kIters / (ms * 1e-3);
    return err;
}
hipError_t launch_diag(const JobDev *jobs, const uint32_t *bprefix, int njobs, uint32_t nblocks, int maxM, hipStream_t st)
{
    if (!nblocks) return hipSuccess;
    if (maxM < 8) hipLaunchKernelGGL(k_diag<8>, dim3(nblocks), dim3(kThreads), 0, st, jobs, bprefix, njobs);
    else if (maxM < 16) hipLaunchKernelGGL(k_diag<16>, dim3(nblocks), dim3(kThreads), 0, st, jobs, bprefix, njobs);
    else hipLaunchKernelGGL(k_diag<65>, dim3(nblocks), dim3(kThreads), 0, st, jobs, bprefix, njobs);
    return hipGetLastError();
}
hipError_t launch_finalize(const JobDev *jobs, const uint32_t *bprefix, int njobs, uint32_t nblocks, int maxM, hipStream_t st)
{
    if (!nblocks) return hipSuccess;
    if (maxM < 8) hipLaunchKernelGGL((k_finalize<8, 1>), dim3(nblocks), dim3(1024), 0, st, jobs, bprefix, njobs);
    else if (maxM < 16) hipLaunchKernelGGL((k_finalize<16, 1>), dim3(nblocks), dim3(1024), 0, st, jobs, bprefix, njobs);
    else hipLaunchKernelGGL((k_finalize<65, 4>), dim3(nblocks), dim3(256), 0, st, jobs, bprefix, njobs);
    return hipGetLastError();
}

}  // namespace gk

namespace gk {
// The row accumulation may keep several levels of a long row in LDS (up to
// the device's per-block limit).
hipError_t init_kernel_attributes(size_t acc_lds)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_accumulate),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)acc_lds);
}
}  // namespace gk
