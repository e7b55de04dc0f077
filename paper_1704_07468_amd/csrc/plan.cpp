// Planning and launch sequence of Gram jobs (host side).
//
// A plan covers one or more jobs.  Every job's position sets ("masks") are
// ordered job by job, level by level; consecutive masks are grouped into
// chunks whose partition and sort buffers fit one reusable pool, and each
// chunk runs count -> scan -> scatter -> sort -> row accumulation before the
// next one reuses the pool.  The int8 matrix-core products, the diagonal and
// the epilogue run once at the end.  Everything the kernels read from the
// host (job and mask descriptors, offsets, coefficient tables, block
// prefixes) travels in one descriptor blob with one copy.
#include "plan.h"

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>

namespace gk {

static thread_local std::string g_err;

void set_error(const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}
const char *last_error() { return g_err.c_str(); }
void clear_error() { g_err.clear(); }
const char *hip_name(hipError_t e) { return hipGetErrorString(e); }

int64_t binom64(int n, int r)
{
    if (r < 0 || n < 0 || r > n) return 0;
    int64_t v = 1;
    for (int i = 1; i <= r; ++i) v = v * (n - r + i) / i;
    return v;
}

int symbol_bits(int sigma)
{
    int b = 0;
    while ((1 << b) < sigma) ++b;
    return b < 1 ? 1 : b;
}

static int ceil_log2(uint64_t x)
{
    int b = 0;
    while ((1ull << b) < x) ++b;
    return b;
}

gakco_status fetch_lens(JobPlan &jp, hipStream_t st)
{
    jp.lens.assign((size_t)jp.N, 0);
    GK_HIP(hipMemcpyAsync(jp.lens.data(), jp.lens_dev, sizeof(int32_t) * (size_t)jp.N, hipMemcpyDeviceToHost, st));
    GK_HIP(hipStreamSynchronize(st));
    return GAKCO_OK;
}

// The kept positions of a mask as runs of consecutive symbol fields.
static MaskDesc make_mask(int g, int b, const int *removed, int m)
{
    MaskDesc md{};
    md.level = m;
    std::vector<char> drop((size_t)g, 0);
    for (int i = 0; i < m; ++i) drop[(size_t)removed[i]] = 1;
    int q = 0, j = 0;
    while (j < g) {
        if (drop[(size_t)j]) { ++j; continue; }
        int L = 0;
        while (j + L < g && !drop[(size_t)(j + L)]) ++L;
        const uint32_t src = (uint32_t)((g - j - L) * b), wid = (uint32_t)(L * b), dst = (uint32_t)((g - m - q - L) * b);
        md.run[md.nrun] = src | wid << 8 | dst << 16;
        md.nrun += 1;
        q += L;
        j += L;
    }
    return md;
}

gakco_status plan_shape(gakco_ctx *ctx, JobPlan &jp, const int32_t *removed_one, int m_one)
{
    if (jp.N < 1) { set_error("N must be >= 1 (got %d)", jp.N); return GAKCO_EINVAL; }
    if (jp.sigma < 1 || jp.sigma > 127) { set_error("sigma must be in 1..127 (got %d)", jp.sigma); return GAKCO_EINVAL; }
    if (jp.g < 1) { set_error("g must be >= 1 (got %d)", jp.g); return GAKCO_EINVAL; }
    if (jp.k < 0 || jp.k > jp.g) { set_error("k must be in 0..g (got k=%d, g=%d)", jp.k, jp.g); return GAKCO_EINVAL; }
    if (!jp.seqs || !jp.lens_dev) { set_error("seqs and lens must not be NULL"); return GAKCO_EINVAL; }
    jp.b = symbol_bits(jp.sigma);
    if (jp.g * jp.b > 64) {
        set_error("g*b = %d*%d exceeds the 64-bit packed g-mer", jp.g, jp.b);
        return GAKCO_EUNSUPPORTED;
    }
    jp.M = jp.g - jp.k;
    const int N = jp.N;
    jp.gstart.assign((size_t)N + 1, 0);
    jp.seq_off.assign((size_t)N + 1, 0);
    uint64_t T = 0;
    uint32_t maxng = 0;
    for (int i = 0; i < N; ++i) {
        const int32_t l = jp.lens[(size_t)i];
        if (l < 0) { set_error("lens[%d] = %d is negative", i, l); return GAKCO_EINVAL; }
        const uint32_t ng = (l >= jp.g) ? (uint32_t)(l - jp.g + 1) : 0u;
        jp.gstart[(size_t)i] = (uint32_t)T;
        jp.seq_off[(size_t)i + 1] = jp.seq_off[(size_t)i] + l;
        T += ng;
        maxng = std::max(maxng, ng);
        if (T >= (1ull << 31)) { set_error("more than 2^31 g-mers"); return GAKCO_EUNSUPPORTED; }
    }
    jp.gstart[(size_t)N] = (uint32_t)T;
    jp.T = (uint32_t)T;
    jp.maxng = maxng;
    jp.nsym = jp.seq_off[(size_t)N];
    jp.sb = std::max(1, ceil_log2((uint64_t)N));
    if (jp.sb > 24 || (uint64_t)maxng >= (1ull << (31 - jp.sb))) {
        set_error("N=%d with %u g-mers in one sequence exceeds the 32-bit run entry", N, maxng);
        return GAKCO_EUNSUPPORTED;
    }
    jp.masks.clear();
    if (removed_one) {
        for (int i = 0; i < m_one; ++i)
            if (removed_one[i] < 0 || removed_one[i] >= jp.g || (i && removed_one[i] <= removed_one[i - 1])) {
                set_error("removed positions must be increasing and in [0, g)");
                return GAKCO_EINVAL;
            }
        jp.masks.push_back(make_mask(jp.g, jp.b, removed_one, m_one));
    } else {
        uint64_t total = 0;
        for (int m = 0; m <= jp.M; ++m) total += (uint64_t)binom64(jp.g, m);
        if (total > (1u << 20)) { set_error("%llu position sets exceed the limit", (unsigned long long)total); return GAKCO_EUNSUPPORTED; }
        // one position set adds at most ng_X * ng_Y to an entry of the row
        // accumulation's uint32 counters; more sets are summed in steps
        if ((uint64_t)maxng * maxng > 0xFFFFFFFFull) {
            set_error("a sequence with %u g-mers exceeds the 32-bit row counters of one position set (limit 65535)", maxng);
            return GAKCO_EUNSUPPORTED;
        }
        for (int m = 0; m <= jp.M; ++m) {
            std::vector<int> P((size_t)m);
            for (int i = 0; i < m; ++i) P[(size_t)i] = i;
            while (true) {
                jp.masks.push_back(make_mask(jp.g, jp.b, P.data(), m));
                int i = m - 1;
                while (i >= 0 && P[(size_t)i] == jp.g - m + i) --i;
                if (i < 0) break;
                P[(size_t)i] += 1;
                for (int q = i + 1; q < m; ++q) P[(size_t)q] = P[(size_t)q - 1] + 1;
            }
        }
    }
    // bucket geometry per level
    jp.level_B.assign((size_t)jp.g + 1, 0);
    for (int m = 0; m <= jp.g; ++m) {
        const int w = (jp.g - m) * jp.b;
        const uint64_t want = (T + (uint64_t)ctx->bucket_avg - 1) / (uint64_t)std::max(1, ctx->bucket_avg);
        int B = ceil_log2(std::max<uint64_t>(1, want));
        const int Bmax = std::min(w, kMaxBucketBits);
        B = std::min(B, Bmax);
        while (w - B + jp.sb > 64 && B < Bmax) ++B;
        if (w - B + jp.sb > 64) { set_error("reduced key + sequence id exceed 64 bits"); return GAKCO_EUNSUPPORTED; }
        jp.level_B[(size_t)m] = B;
    }
    jp.Npad = (N + 63) / 64 * 64;
    return GAKCO_OK;
}

// Device buffers of one mask inside the pool: bucket offsets and cursors,
// the bucketed (composite, index) pairs and their ping-pong copies, the run
// entries and the per-g-mer info.
struct MaskBuf {
    size_t boff, bcur, comp, idx, comp2, idx2, E, info, size;
};
static MaskBuf mask_buf(uint32_t T, int B)
{
    Layout l;
    const size_t nb = (size_t)1 << B;
    MaskBuf m{};
    m.boff = l.take((nb + 1) * 4);
    m.bcur = l.take(nb * 4);
    m.comp = l.take((size_t)T * 8);
    m.idx = l.take((size_t)T * 4);
    m.comp2 = l.take((size_t)T * 8);
    m.idx2 = l.take((size_t)T * 4);
    m.E = l.take((size_t)T * 4);
    m.info = l.take((size_t)T * 8);
    m.size = l.size;
    return m;
}

static int job_tau(const gakco_ctx *ctx, const JobPlan &jp) { return jp.tau >= 0 ? jp.tau : ctx->dense_tau; }

// Rows [r0, r1) of each split, as split_range computes them on the device:
// the largest split's row count for R rows over at most S splits.
static uint32_t split_rows_max(uint32_t R, int S)
{
    const uint32_t used = std::max(1u, std::min((uint32_t)S, (R + kDenseMinSplitRows - 1) / kDenseMinSplitRows));
    return ((R + used - 1) / used + (uint32_t)kDenseK - 1) / (uint32_t)kDenseK * (uint32_t)kDenseK;
}

// Which levels of a job are grouped by direct addressing (no sort): those
// whose reduced g-mers take at most kDirectMaxKeys values, whose int8
// products stay exact in int32 per row split, and -- in the automatic mode
// -- whose modelled time (count-matrix products and writes) beats that of
// sorting the level and updating its groups pair by pair (or as count rows
// when they are dense anyway).  Moves the position sets of those levels
// from jp.masks to jp.dmasks.
static void plan_direct(const gakco_ctx *ctx, JobPlan &jp)
{
    const int M1 = jp.M + 1;
    jp.direct.assign((size_t)M1, 0);
    jp.dKp.assign((size_t)M1, 0);
    jp.dR.assign((size_t)M1, 0);
    jp.dstride.assign((size_t)M1, 0);
    jp.dSd.assign((size_t)M1, 0);
    jp.o_Dd.assign((size_t)M1, 0);
    jp.o_Pd.assign((size_t)M1, 0);
    if (!jp.dmasks.empty()) {  // planned before: restore the level order
        jp.masks.insert(jp.masks.end(), jp.dmasks.begin(), jp.dmasks.end());
        std::stable_sort(jp.masks.begin(), jp.masks.end(),
                         [](const MaskDesc &a, const MaskDesc &b) { return a.level < b.level; });
        jp.dmasks.clear();
    }
    if (ctx->direct_mode == 0 || !jp.want_kernel || !jp.ext_boff.empty() || !jp.ext_diag.empty() || jp.T == 0) return;
    const int ntile = jp.Ntile / dense_tile();
    const int tiles = ntile * (ntile + 1) / 2;
    const double sq = (double)jp.maxng * (double)jp.maxng;
    const double T = (double)jp.T, Nt = (double)jp.Ntile;
    const int tau = job_tau(ctx, jp);
    // measured rates on MI355X: ~30 ps per (position set, g-mer) through the
    // partition and sort, ~8e11 pair updates/s in the row accumulation,
    // ~5e14 int8 MACs/s in the count-matrix products, ~5e12 B/s of row writes
    constexpr double kSortS = 3.0e-11, kUpd = 8.0e11, kMac = 5.0e14, kWrite = 5.0e12;
    size_t bytes = 0;
    for (int m = 0; m <= jp.M; ++m) {
        uint64_t K = 1;
        bool small = true;
        for (int q = 0; q < jp.g - m && small; ++q) {
            K *= (uint64_t)jp.sigma;
            small = K <= kDirectMaxKeys;
        }
        if (!small) continue;
        const uint64_t Kp = (K + 15) / 16 * 16;
        const uint64_t nm = (uint64_t)binom64(jp.g, m);
        const uint64_t R = nm * Kp;
        if (R >= (1ull << 31)) continue;
        // splits: about 1024 blocks of products, each split's int32 sums exact
        // (at most 65536 rows of counts <= 127, or few enough position sets:
        // one adds at most ng_X * ng_Y to an entry)
        int S = std::max(1, std::min(kDenseMaxSplits, (1024 + tiles - 1) / tiles));
        auto exact = [&](int s) {
            const uint32_t per = split_rows_max((uint32_t)R, s);
            return per <= kDenseSplitRows || ((double)(per / Kp + 2) * sq < 2147483647.0);
        };
        while (!exact(S) && S < kDenseMaxSplits) ++S;
        if (!exact(S)) continue;
        const double t_direct = (double)Kp * Nt * Nt * 0.5 / kMac + (double)Kp * Nt / kWrite;
        const double lam = T / (double)K;  // g-mers per reduced g-mer
        const double t_sort = T * kSortS + (tau > 0 && lam >= tau ? (double)K * Nt * Nt * 0.5 / kMac : T * lam * 0.5 / kUpd);
        if (ctx->direct_mode == 1 && t_direct >= t_sort) continue;
        const uint64_t stride = (R + 63) / 64 * 64;
        const size_t lb = (size_t)jp.Ntile * stride + (size_t)tiles * S * dense_tile() * dense_tile() * 4;
        if (bytes + lb > ctx->budget / 4) continue;
        bytes += lb;
        jp.direct[(size_t)m] = 1;
        jp.dKp[(size_t)m] = (uint32_t)Kp;
        jp.dR[(size_t)m] = (uint32_t)R;
        jp.dstride[(size_t)m] = (uint32_t)stride;
        jp.dSd[(size_t)m] = S;
    }
    std::vector<MaskDesc> keep;
    for (auto &md : jp.masks) (jp.direct[(size_t)md.level] ? jp.dmasks : keep).push_back(md);
    jp.masks.swap(keep);
}

gakco_status plan_layout(gakco_ctx *ctx, Plan &p)
{
    Layout &L = p.lay;
    L = Layout{};
    p.output_bytes = 0;
    p.dense_bytes = 0;
    p.n_dense = 0;
    p.maxM = 0;
    p.pool_bytes = 0;
    p.chunks.clear();
    p.n_dlev = p.n_dwork = p.n_dchunk = 0;
    p.dclass.clear();
    p.excess_cap = 0;
    p.excess_overflow = false;
    size_t nmask = 0;
    p.nflags = p.jobs.size();
    for (auto &jp : p.jobs) {
        const size_t N = (size_t)jp.N, M1 = (size_t)jp.M + 1;
        jp.Ntile = (jp.N + dense_tile() - 1) / dense_tile() * dense_tile();
        plan_direct(ctx, jp);
        if (!jp.key_override) {
            jp.o_key = L.take((size_t)jp.T * 8);
            jp.o_sid = L.take((size_t)jp.T * 4);
        }
        jp.mask_first = (int)nmask;
        nmask += jp.masks.size();
        jp.lev_base = p.nflags - p.jobs.size();
        p.nflags += M1;
        jp.dcap.assign(M1, 0);
        jp.o_dense.assign(M1, 0);
        jp.o_P.assign(M1, 0);
        if (!jp.want_kernel) continue;
        // row slabs: a block of the row accumulation keeps one slab of a
        // row's int32 counters in LDS
        {
            const int cap = (int)std::min<size_t>(ctx->lds_max / 4 / 64 * 64, (size_t)1 << 20);
            if (cap < 64) { set_error("no LDS for the row accumulation"); return GAKCO_EUNSUPPORTED; }
            int S = jp.Npad;
            if (ctx->acc_slab > 0) S = std::min(S, ctx->acc_slab);
            jp.acc_slab = std::min(S, cap);
            jp.acc_nslab = (jp.N + jp.acc_slab - 1) / jp.acc_slab;
        }
        jp.own_C = !jp.Cm_out && !jp.Nm_out;
        if (jp.own_C) jp.o_C = L.take(M1 * N * N * 8);
        jp.o_Kd = L.take(N * 8);
        p.output_bytes += N * N * 8 * ((jp.K_out ? 1 : 0) + (jp.Nm_out ? M1 : 0) + (jp.Cm_out ? M1 : 0));
        p.maxM = std::max(p.maxM, jp.M);
        // int8 matrix-core path: per level a sequence-major count matrix in
        // the context's dense buffer, its capacity bounded by how many groups
        // can have tau distinct sequences; rows are split over dS blocks per
        // output tile so that about 1024 blocks run, a split holding at most
        // 65536 rows so that its int32 partial sums stay exact
        const int tau = job_tau(ctx, jp);
        if (tau > 0 && !jp.masks.empty()) {
            const size_t limit = std::min<size_t>(ctx->budget / 8, 8ull << 30);
            std::vector<double> want(M1, 0.0);
            double tot = 0;
            for (int m = 0; m <= jp.M; ++m) {
                want[(size_t)m] = (double)binom64(jp.g, m) * ((double)jp.T / tau + 1.0);
                tot += want[(size_t)m] * jp.Ntile;
            }
            const double scale = tot > (double)limit ? (double)limit / tot : 1.0;
            const int ntile = jp.Ntile / dense_tile();
            const int tiles = ntile * (ntile + 1) / 2;
            jp.dS = std::max(1, std::min(kDenseMaxSplits, (1024 + tiles - 1) / tiles));
            // a fixed scratch keeps one split per tile and the partial tiles of
            // the heaviest levels (highest m first) within a quarter of it
            if (ctx->fixed_arena) jp.dS = 1;
            size_t part_left = ctx->fixed_arena ? ctx->budget / 4 : ~(size_t)0;
            const size_t part_bytes = (size_t)tiles * dense_tile() * dense_tile() * 4;
            const uint64_t kc = (uint64_t)dense_kchunk();
            for (int m = jp.M; m >= 0; --m) {
                if (jp.direct[(size_t)m]) continue;
                uint64_t c = (uint64_t)(want[(size_t)m] * scale);
                c = std::min<uint64_t>(c, (uint64_t)jp.dS * dense_split_rows());
                c = c / kc * kc;
                if (c < kc) continue;
                if (part_bytes * (size_t)jp.dS > part_left) continue;
                part_left -= part_bytes * (size_t)jp.dS;
                jp.dcap[(size_t)m] = (uint32_t)c;
                jp.o_dense[(size_t)m] = p.dense_bytes;
                p.dense_bytes += (size_t)jp.Ntile * c;
                jp.o_P[(size_t)m] = L.take((size_t)tiles * jp.dS * dense_tile() * dense_tile() * 4);
                p.n_dense += 1;
            }
        }
        // direct-address levels: count matrix and split partial tiles
        {
            const int ntile = jp.Ntile / dense_tile();
            const size_t tiles = (size_t)ntile * (ntile + 1) / 2;
            for (int m = 0; m <= jp.M; ++m) {
                if (!jp.direct[(size_t)m]) continue;
                jp.o_Dd[(size_t)m] = L.take((size_t)jp.Ntile * jp.dstride[(size_t)m]);
                jp.o_Pd[(size_t)m] = L.take(tiles * (size_t)jp.dSd[(size_t)m] * dense_tile() * dense_tile() * 4);
                p.n_dlev += 1;
                p.n_dchunk += (int)((binom64(jp.g, m) + kDirectMasksPerBlock - 1) / kDirectMasksPerBlock);
            }
            p.n_dwork += (int)jp.dmasks.size();
        }
    }
    // counts above 127 in directly addressed position sets (their counter is
    // the last flag word)
    p.f_excess = p.nflags;
    p.nflags += 1;
    {
        // a sequence with ng g-mers has at most ng / 128 reduced g-mers counted
        // more than 127 times in one position set
        uint64_t bound = 0;
        for (auto &jp : p.jobs) {
            if (jp.dmasks.empty()) continue;
            uint64_t q = 0;
            for (int X = 0; X < jp.N; ++X) q += (jp.gstart[(size_t)X + 1] - jp.gstart[(size_t)X]) >> 7;
            bound += q * jp.dmasks.size();
        }
        p.excess_cap = (uint32_t)std::min<uint64_t>(bound, ctx->excess_cap ? ctx->excess_cap : kExcessCap);
    }
    p.o_excess = L.take((size_t)std::max(1u, p.excess_cap) * 16);
    p.mw.assign(nmask, MaskWork{});
    p.o_flags = L.take(p.nflags * 4);
    // chunks: greedy runs of masks whose buffers fit the pool
    const size_t outb = ctx->fixed_arena ? 0 : p.output_bytes;  // caller outputs outside a fixed scratch
    const size_t fixed = L.size + (16u << 20);  // + descriptor headroom
    const size_t reserved = fixed + p.dense_bytes + outb;
    if (reserved >= ctx->budget) {
        set_error("scratch %.3f GB + count matrices %.3f GB + outputs %.3f GB exceed the %s %.3f GB", fixed / 1e9,
                  p.dense_bytes / 1e9, outb / 1e9, ctx->fixed_arena ? "fixed scratch of" : "HBM budget",
                  ctx->budget / 1e9);
        return GAKCO_EBUDGET;
    }
    const size_t pool_limit = std::min(ctx->budget - reserved, ctx->pool_cap);
    {
        Chunk cur;
        Layout pl;
        size_t nbc = 0;
        auto close = [&]() {
            if (!cur.nmask) return;
            cur.nbuck = nbc;
            cur.nbcnt = nbc + kSortCounters;
            cur.o_bcnt = pl.take(cur.nbcnt * 4);
            cur.o_lists = pl.take((size_t)kSortClasses * nbc * 4);
            p.pool_bytes = std::max(p.pool_bytes, pl.size);
            p.chunks.push_back(cur);
            cur = Chunk{};
            pl = Layout{};
            nbc = 0;
        };
        int gi = 0;
        for (auto &jp : p.jobs) {
            for (size_t i = 0; i < jp.masks.size(); ++i, ++gi) {
                const int B = jp.level_B[(size_t)jp.masks[i].level];
                const MaskBuf mb = mask_buf(jp.T, B);
                const size_t need = mb.size + ((size_t)4 << B) * (1 + kSortClasses) + 512;
                if (need > pool_limit) {
                    set_error("one position set needs %.3f GB of buffers; %.3f GB of the HBM budget are left",
                              need / 1e9, pool_limit / 1e9);
                    return GAKCO_EBUDGET;
                }
                if (cur.nmask && pl.size + need + nbc * 4 * (1 + kSortClasses) + 4 * kSortCounters + 512 > pool_limit) close();
                if (ctx->chunk_masks > 0 && cur.nmask >= ctx->chunk_masks) close();
                if (cur.nmask >= kMaxChunkMasks) close();  // the sort lists' mask field
                if (!cur.nmask) cur.mfirst = gi;
                cur.o_mask.push_back(pl.take(mb.size));
                cur.nmask += 1;
                cur.maxB = std::max(cur.maxB, B);
                nbc += (size_t)1 << B;
            }
        }
        close();
    }
    // accumulation works of each chunk: one per (job, level) present in it,
    // the levels with the most masks first; the first work of a (job, level)
    // stores its rows, later ones add to them
    std::vector<std::vector<char>> stored(p.jobs.size());
    for (size_t j = 0; j < p.jobs.size(); ++j) stored[j].assign((size_t)p.jobs[j].M + 1, 0);
    for (auto &c : p.chunks) {
        for (size_t j = 0; j < p.jobs.size(); ++j) {
            auto &jp = p.jobs[j];
            if (!jp.want_kernel) continue;
            const int a = std::max(c.mfirst, jp.mask_first);
            const int b = std::min(c.mfirst + c.nmask, jp.mask_first + (int)jp.masks.size());
            for (int lev = jp.M; lev >= 0; --lev) {
                int first = -1, cnt = 0;
                for (int gi = a; gi < b; ++gi)
                    if (jp.masks[(size_t)(gi - jp.mask_first)].level == lev) {
                        if (first < 0) first = gi;
                        ++cnt;
                    }
                if (!cnt) continue;
                AccWork w{};
                w.job = (int)j;
                w.mfirst = first;
                w.nmask = cnt;
                w.level = lev;
                w.Npad = jp.acc_slab;
                w.slab = jp.acc_slab;
                w.nslab = jp.acc_nslab;
                w.first = stored[j][(size_t)lev] ? 0 : 1;
                stored[j][(size_t)lev] = 1;
                // masks per flush of the uint32 row: mstep * maxng^2 < 2^32
                {
                    const uint64_t sq = std::max<uint64_t>(1, (uint64_t)jp.maxng * jp.maxng);
                    w.mstep = (int)std::min<uint64_t>((uint64_t)cnt, std::max<uint64_t>(1, 0xFFFFFFFFull / sq));
                    if (ctx->acc_mstep > 0) w.mstep = std::min(w.mstep, ctx->acc_mstep);
                }
                c.aw.push_back(w);
                c.acc_lds = std::max(c.acc_lds, (size_t)jp.acc_slab * 4);
            }
        }
        c.nacc = (int)c.aw.size();
    }
    // descriptor blob
    Layout d;
    const size_t nj = p.jobs.size();
    p.d_jobs = d.take(sizeof(JobDev) * nj, 64);
    p.d_masks = d.take(sizeof(MaskWork) * std::max<size_t>(1, nmask), 64);
    p.d_dense = d.take(dense_work_size() * (size_t)std::max(1, p.n_dense + p.n_dlev), 64);
    p.d_pdense = d.take(((size_t)p.n_dense + p.n_dlev + 1) * 4, 64);
    p.d_pdtile = d.take(((size_t)p.n_dense + p.n_dlev + 1) * 4, 64);
    p.d_dlev = d.take(sizeof(DirectLevel) * (size_t)std::max(1, p.n_dlev), 64);
    p.d_dwork = d.take(sizeof(DirectWork) * (size_t)std::max(1, p.n_dwork), 64);
    p.d_dchunk = d.take(8 * (size_t)std::max(1, p.n_dchunk), 64);
    p.d_pdir = d.take(((size_t)p.n_dchunk + 32) * 4, 64);
    p.d_drows = d.take((size_t)std::max(1, p.n_dlev) * 4, 64);
    p.d_pv = d.take((nj + 1) * 4, 64);
    p.d_px = d.take((nj + 1) * 4, 64);
    p.d_pd = d.take((nj + 1) * 4, 64);
    p.d_pf = d.take((nj + 1) * 4, 64);
    for (auto &jp : p.jobs) {
        const size_t M1 = (size_t)jp.M + 1;
        jp.o_seqoff = d.take(((size_t)jp.N + 1) * 8, 64);
        jp.o_gstart = d.take(((size_t)jp.N + 1) * 4, 64);
        jp.o_coef = d.take(M1 * M1 * 8, 64);
        jp.o_hco = d.take(M1 * 8, 64);
        jp.o_dref = d.take(M1 * sizeof(DenseRef), 64);
    }
    for (auto &c : p.chunks) {
        c.d_pt = d.take(((size_t)c.nmask + 1) * 4, 64);
        c.d_ptc = d.take(((size_t)c.nmask + 1) * 4, 64);
        c.d_acc = d.take(sizeof(AccWork) * (size_t)std::max(1, c.nacc), 64);
        c.d_pacc = d.take(((size_t)c.nacc + 1) * 4, 64);
    }
    p.desc_bytes = d.size;
    p.o_pool = L.take(p.pool_bytes);
    p.o_desc = L.take(p.desc_bytes);
    if (L.size + (ctx->fixed_arena ? 256 : 0) + p.dense_bytes + outb > ctx->budget) {
        set_error("scratch %.3f GB + count matrices %.3f GB + outputs %.3f GB exceed the %s %.3f GB", L.size / 1e9,
                  p.dense_bytes / 1e9, outb / 1e9, ctx->fixed_arena ? "fixed scratch of" : "HBM budget",
                  ctx->budget / 1e9);
        return GAKCO_EBUDGET;
    }
    return GAKCO_OK;
}

gakco_status ctx_small_buffer(gakco_ctx *ctx, void **out)
{
    if (!ctx->small) {
        if (ctx->fixed_arena) { set_error("no small buffer in a fixed-scratch call"); return GAKCO_EINVAL; }
        GK_HIP(hipMalloc(&ctx->small, 4096));
    }
    *out = ctx->small;
    return GAKCO_OK;
}

static gakco_status reserve_arena(gakco_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->arena_cap) return GAKCO_OK;
    if (ctx->fixed_arena) {
        set_error("the call needs %zu bytes of scratch; the fixed scratch holds %zu", bytes, ctx->arena_cap);
        return GAKCO_EBUDGET;
    }
    if (ctx->arena) {
        GK_HIP(hipDeviceSynchronize());
        GK_HIP(hipFree(ctx->arena));
        ctx->arena = nullptr;
        ctx->arena_cap = 0;
    }
    const size_t cap = (bytes + (64ull << 20) - 1) / (64ull << 20) * (64ull << 20);
    GK_HIP(hipMalloc(&ctx->arena, cap));
    ctx->arena_cap = cap;
    return GAKCO_OK;
}

static uint32_t uniform_of(const std::vector<uint32_t> &pre)
{
    if (pre.size() < 2) return 0;
    const uint32_t u = pre[1] - pre[0];
    for (size_t i = 1; i < pre.size(); ++i)
        if (pre[i] - pre[i - 1] != u) return 0;
    return u;
}

gakco_status plan_bind(gakco_ctx *ctx, Plan &p, hipStream_t st)
{
    GK_TRY(reserve_arena(ctx, p.lay.size));
    if (ctx->fixed_arena) {
        // count matrices after the arena's layout, cleared by every call (the
        // region is shared with calls of other shapes)
        const size_t off = (p.lay.size + 255) / 256 * 256;
        if (off + p.dense_bytes > ctx->arena_cap) {
            set_error("scratch %zu + count matrices %zu bytes exceed the fixed scratch of %zu", off, p.dense_bytes,
                      ctx->arena_cap);
            return GAKCO_EBUDGET;
        }
        ctx->dense_buf = p.dense_bytes ? reinterpret_cast<int8_t *>(ctx->arena) + off : nullptr;
        ctx->dense_cap = p.dense_bytes;
        ctx->dense_dirty = p.dense_bytes > 0;
    } else if (p.dense_bytes > ctx->dense_cap) {
        if (ctx->dense_buf) {
            GK_HIP(hipDeviceSynchronize());
            GK_HIP(hipFree(ctx->dense_buf));
            ctx->dense_buf = nullptr;
            ctx->dense_cap = 0;
        }
        GK_HIP(hipMalloc(&ctx->dense_buf, p.dense_bytes));
        ctx->dense_cap = p.dense_bytes;
        ctx->dense_dirty = true;
    }
    if (ctx->dense_dirty && ctx->dense_buf) {
        GK_HIP(launch_fill_u64(reinterpret_cast<uint64_t *>(ctx->dense_buf), ctx->dense_cap / 8, 0ull, st));
        ctx->dense_dirty = false;
    }
    char *base = (char *)ctx->arena;
    p.base = base;
    char *dev_desc = base + p.o_desc;
    char *pool = base + p.o_pool;
    uint32_t *flags = reinterpret_cast<uint32_t *>(base + p.o_flags);
    p.desc_host.assign(p.desc_bytes, 0);
    char *blob = p.desc_host.data();
    auto put = [&](size_t off, const std::vector<uint32_t> &v) { memcpy(blob + off, v.data(), v.size() * 4); };
    JobDev *jd = reinterpret_cast<JobDev *>(blob + p.d_jobs);
    std::vector<uint32_t> pv(1, 0), px(1, 0), pd(1, 0), pf(1, 0), pdn(1, 0), pdt(1, 0);
    struct HostChunk {
        uint32_t w0, nw, kp, ntile;
    };
    std::vector<HostChunk> hchunks;
    int di = 0, dl_next = 0, dw_next = 0;
    DirectLevel *dlev = reinterpret_cast<DirectLevel *>(blob + p.d_dlev);
    DirectWork *dwork = reinterpret_cast<DirectWork *>(blob + p.d_dwork);
    uint32_t *drows = reinterpret_cast<uint32_t *>(blob + p.d_drows);
    for (size_t j = 0; j < p.jobs.size(); ++j) {
        auto &jp = p.jobs[j];
        const int M1 = jp.M + 1;
        // host tables into the blob
        memcpy(blob + jp.o_seqoff, jp.seq_off.data(), jp.seq_off.size() * 8);
        memcpy(blob + jp.o_gstart, jp.gstart.data(), jp.gstart.size() * 4);
        int64_t *coef = reinterpret_cast<int64_t *>(blob + jp.o_coef);
        int64_t *hco = reinterpret_cast<int64_t *>(blob + jp.o_hco);
        for (int m = 0; m < M1; ++m) {
            hco[m] = binom64(jp.g - m, jp.k);                                                 // Eq. 6
            for (int q = 0; q < m; ++q) coef[(size_t)m * M1 + q] = binom64(jp.g - q, m - q);  // Eq. 9
        }
        DenseRef *dref = reinterpret_cast<DenseRef *>(blob + jp.o_dref);
        std::vector<int> dl_of((size_t)M1, -1);
        for (int m = 0; m < M1; ++m) {
            dref[m] = DenseRef{};
            if (jp.want_kernel && jp.direct[(size_t)m]) {
                dref[m].P = reinterpret_cast<const int32_t *>(p.base + jp.o_Pd[(size_t)m]);
                dref[m].count = reinterpret_cast<const uint32_t *>(dev_desc + p.d_drows) + dl_next;
                dref[m].cap = jp.dR[(size_t)m];
                dref[m].S = jp.dSd[(size_t)m];
                dref[m].ntile = jp.Ntile / dense_tile();
                dl_of[(size_t)m] = dl_next++;
            } else if (jp.want_kernel && jp.dcap[(size_t)m]) {
                dref[m].P = reinterpret_cast<const int32_t *>(p.base + jp.o_P[(size_t)m]);
                dref[m].count = reinterpret_cast<const uint32_t *>(p.base + p.o_flags) + p.jobs.size() + jp.lev_base + m;
                dref[m].cap = jp.dcap[(size_t)m];
                dref[m].S = jp.dS;
                dref[m].ntile = jp.Ntile / dense_tile();
            }
        }
        JobDev &J = jp.dev;
        J = JobDev{};
        J.seqs = jp.seqs;
        J.seq_off = reinterpret_cast<const int64_t *>(dev_desc + jp.o_seqoff);
        J.gstart = reinterpret_cast<const uint32_t *>(dev_desc + jp.o_gstart);
        J.N = jp.N; J.sigma = jp.sigma; J.g = jp.g; J.k = jp.k; J.M = jp.M; J.b = jp.b; J.sb = jp.sb;
        J.T = jp.T;
        J.nsym = jp.nsym;
        J.key = jp.key_override ? jp.key_override : reinterpret_cast<uint64_t *>(base + jp.o_key);
        J.kshift = (!jp.key_override && jp.g * jp.b < 64 && jp.g * jp.b + jp.sb <= 64) ? jp.g * jp.b : 0;
        J.sid = jp.sid_override ? jp.sid_override : reinterpret_cast<uint32_t *>(base + jp.o_sid);
        J.err = reinterpret_cast<int32_t *>(flags + j);
        if (jp.want_kernel) {
            J.C = jp.own_C ? reinterpret_cast<int64_t *>(base + jp.o_C) : (jp.Cm_out ? jp.Cm_out : jp.Nm_out);
            J.Kd = reinterpret_cast<int64_t *>(base + jp.o_Kd);
            J.coef = reinterpret_cast<const int64_t *>(dev_desc + jp.o_coef);
            J.hco = reinterpret_cast<const int64_t *>(dev_desc + jp.o_hco);
            J.dref = reinterpret_cast<const DenseRef *>(dev_desc + jp.o_dref);
            J.K_out = jp.K_out;
            J.Nm_out = jp.Nm_out;
            J.Cm_out = jp.Cm_out;
        }
        jd[j] = J;
        for (int m = 0; m < M1; ++m) {
            const int dl = dl_of[(size_t)m];
            if (dl < 0) continue;
            DirectLevel &L = dlev[dl];
            L = DirectLevel{};
            L.D = reinterpret_cast<int8_t *>(base + jp.o_Dd[(size_t)m]);
            L.stride = jp.dstride[(size_t)m];
            L.R = jp.dR[(size_t)m];
            L.Kp = jp.dKp[(size_t)m];
            L.job = (int)j;
            L.level = m;
            L.nd = jp.g - m;
            L.b = jp.b;
            L.sigma = jp.sigma;
            L.pow2 = (1 << jp.b) == jp.sigma ? 1 : 0;
            drows[dl] = L.R;
            uint32_t row0 = 0;
            for (size_t q = 0; q < jp.dmasks.size(); ++q) {
                if (jp.dmasks[q].level != m) continue;
                if (row0 / L.Kp % kDirectMasksPerBlock == 0)
                    hchunks.push_back(HostChunk{(uint32_t)dw_next, 0u, L.Kp, (uint32_t)jp.Ntile});
                hchunks.back().nw += 1;
                DirectWork &W = dwork[dw_next++];
                W = DirectWork{};
                W.md = jp.dmasks[q];
                W.dl = dl;
                W.row0 = row0;
                W.first = row0 == 0 ? 1 : 0;
                row0 += L.Kp;
                W.last = row0 == L.R ? 1 : 0;
            }
        }
        pv.push_back(pv.back() + (uint32_t)((jp.nsym + kThreads * 16 - 1) / (kThreads * 16)));
        px.push_back(px.back() + (jp.T + kThreads - 1) / kThreads);
        pd.push_back(pd.back() + (jp.want_kernel ? (uint32_t)((jp.N + kThreads - 1) / kThreads) : 0u));
        const uint32_t nt = (uint32_t)((jp.N + 31) / 32);
        pf.push_back(pf.back() + (jp.want_kernel ? nt * (nt + 1) / 2 : 0u));  // upper tiles
        if (jp.want_kernel) {
            const int ntile = jp.Ntile / dense_tile();
            const uint32_t tiles = (uint32_t)(ntile * (ntile + 1) / 2);
            for (int m = 0; m <= jp.M; ++m) {
                if (!jp.dcap[(size_t)m]) continue;
                dense_work_fill(blob + p.d_dense + dense_work_size() * (size_t)di, ctx->dense_buf + jp.o_dense[(size_t)m],
                                flags + p.jobs.size() + jp.lev_base + m, jp.dcap[(size_t)m], jp.dcap[(size_t)m], jp.N,
                                ntile, jp.dS, reinterpret_cast<int32_t *>(base + jp.o_P[(size_t)m]));
                pdn.push_back(pdn.back() + tiles * (uint32_t)jp.dS);
                pdt.push_back(pdt.back() + tiles);
                ++di;
            }
        }
    }
    // the direct levels' int8 products come after every sort-path count
    // matrix (only those are cleared after use)
    for (size_t j = 0; j < p.jobs.size(); ++j) {
        auto &jp = p.jobs[j];
        if (!jp.want_kernel) continue;
        const int ntile = jp.Ntile / dense_tile();
        const uint32_t tiles = (uint32_t)(ntile * (ntile + 1) / 2);
        for (int m = 0; m <= jp.M; ++m) {
            if (!jp.direct[(size_t)m]) continue;
            const DenseRef &R = reinterpret_cast<const DenseRef *>(blob + jp.o_dref)[m];
            dense_work_fill(blob + p.d_dense + dense_work_size() * (size_t)di,
                            reinterpret_cast<int8_t *>(base + jp.o_Dd[(size_t)m]), R.count, jp.dR[(size_t)m],
                            jp.dstride[(size_t)m], jp.N, ntile, jp.dSd[(size_t)m],
                            reinterpret_cast<int32_t *>(base + jp.o_Pd[(size_t)m]));
            pdn.push_back(pdn.back() + tiles * (uint32_t)jp.dSd[(size_t)m]);
            pdt.push_back(pdt.back() + tiles);
            ++di;
        }
    }
    // row-writer chunks by counter-array size (powers of two, largest
    // first), one launch each, so that a launch's LDS fits its chunks
    {
        auto cls = [](uint32_t kp) {
            int c = 0;
            while ((1u << c) < kp) ++c;
            return c;
        };
        std::stable_sort(hchunks.begin(), hchunks.end(),
                         [&](const HostChunk &a, const HostChunk &b) { return cls(a.kp) > cls(b.kp); });
        uint2 *ch = reinterpret_cast<uint2 *>(blob + p.d_dchunk);
        uint32_t *pre = reinterpret_cast<uint32_t *>(blob + p.d_pdir);
        size_t pre_used = 0;
        for (size_t i = 0; i < hchunks.size();) {
            size_t e = i;
            Plan::DirClass dc;
            dc.first = (int)i;
            dc.kp = 1u << cls(hchunks[i].kp);
            std::vector<uint32_t> pr(1, 0);
            while (e < hchunks.size() && cls(hchunks[e].kp) == cls(hchunks[i].kp)) {
                ch[e] = make_uint2(hchunks[e].w0, hchunks[e].nw);
                pr.push_back(pr.back() + hchunks[e].ntile);
                ++e;
            }
            dc.nchunk = (int)(e - i);
            dc.d_pre = p.d_pdir + pre_used * 4;
            memcpy(pre + pre_used, pr.data(), pr.size() * 4);
            pre_used += pr.size();
            dc.nblocks = pr.back();
            dc.uniform = uniform_of(pr);
            p.dclass.push_back(dc);
            i = e;
        }
    }
    // mask works, chunk by chunk (each chunk's buffers at the start of the pool)
    size_t j = 0;
    for (auto &c : p.chunks) {
        size_t bc = 0;
        std::vector<uint32_t> pt(1, 0), ptc(1, 0);
        uint64_t bound_big = 0, bound_block = 0, bound_gpk = 0, bound_gwide = 0;
        for (int q = 0; q < c.nmask; ++q) {
            const int gi = c.mfirst + q;
            while (gi >= p.jobs[j].mask_first + (int)p.jobs[j].masks.size()) ++j;
            auto &jp = p.jobs[j];
            const MaskDesc &md = jp.masks[(size_t)(gi - jp.mask_first)];
            MaskWork &W = p.mw[(size_t)gi];
            W = MaskWork{};
            W.md = md;
            W.job = (int)j;
            W.T = jp.T;
            W.N = jp.N;
            const int m = md.level;
            W.w = (jp.g - m) * jp.b;
            W.B = jp.level_B[(size_t)m];
            W.hb = W.w - W.B;
            W.sb = jp.sb;
            W.cb = W.hb + W.sb;
            W.ib = std::max(1, ceil_log2((uint64_t)jp.T + 1));
            W.key = jp.dev.key;
            W.kshift = jp.dev.kshift;
            W.sid = jp.dev.sid;
            const size_t nb = (size_t)1 << W.B;
            W.bcnt = reinterpret_cast<uint32_t *>(pool + c.o_bcnt) + bc;
            bc += nb;
            const MaskBuf mb = mask_buf(jp.T, W.B);
            char *mbp = pool + c.o_mask[(size_t)q];
            W.boff = reinterpret_cast<uint32_t *>(mbp + mb.boff);
            W.bcur = reinterpret_cast<uint32_t *>(mbp + mb.bcur);
            W.comp = reinterpret_cast<uint64_t *>(mbp + mb.comp);
            W.idx = reinterpret_cast<uint32_t *>(mbp + mb.idx);
            W.comp2 = reinterpret_cast<uint64_t *>(mbp + mb.comp2);
            W.idx2 = reinterpret_cast<uint32_t *>(mbp + mb.idx2);
            W.E = reinterpret_cast<uint32_t *>(mbp + mb.E);
            W.info = reinterpret_cast<uint2 *>(mbp + mb.info);
            const size_t mi = (size_t)(gi - jp.mask_first);
            if (!jp.ext_boff.empty()) {
                W.boff = jp.ext_boff[mi];
                W.bgrp = jp.ext_bgrp[mi];
                W.E = jp.ext_E[mi];
                W.gtab = jp.ext_gtab[mi];
            }
            if (!jp.ext_diag.empty()) W.diag = jp.ext_diag[(size_t)m];
            W.inl = jp.want_kernel ? 1 : 0;
            W.i4 = (jp.want_kernel && ctx->info4 && jp.T <= kInfo4MaxT && jp.sb <= 12) ? 1 : 0;
            if (jp.want_kernel && jp.dcap[(size_t)m]) {
                W.D = ctx->dense_buf + jp.o_dense[(size_t)m];
                W.dcount = flags + p.jobs.size() + jp.lev_base + m;
                W.dcap = jp.dcap[(size_t)m];
                W.dstride = jp.dcap[(size_t)m];
                W.tau = job_tau(ctx, jp);
            }
            pt.push_back(pt.back() + (jp.T + kTile - 1) / kTile);
            ptc.push_back(ptc.back() + (jp.T + kCountTile - 1) / kCountTile);
        }
        // grids of the per-bucket sort: at most T / (class minimum) buckets
        // of a mask fall in the block and global classes
        for (int q = 0; q < c.nmask; ++q) {
            const MaskWork &W = p.mw[(size_t)(c.mfirst + q)];
            const bool pk = W.cb + W.ib <= 64;
            bound_big += W.T / ((pk ? kSortWaveMaxPk : kSortWaveMaxWide) / 2 + 1);
            bound_block += W.T / ((pk ? kSortWaveMaxPk : kSortWaveMaxWide) + 1);
            if (pk) bound_gpk += W.T / (kSortBlockMaxPk + 1);
            else bound_gwide += W.T / (kSortBlockMaxWide + 1);
        }
        // one wave per bucket up to 65536 blocks (the class lists put the
        // largest buckets first, so the first waves take the longest work);
        // a persistent grid of 2048 blocks left its slowest waves as a tail
        c.sgrid.wave_blocks = (uint32_t)std::min<size_t>((c.nbuck + kWaves - 1) / kWaves, 65536);
        c.sgrid.wave_big_blocks = (uint32_t)std::min<uint64_t>((bound_big + kWaves - 1) / kWaves, 65536);
        c.sgrid.block_blocks = (uint32_t)std::min<uint64_t>(bound_block, 256);
        c.sgrid.global_blocks_pk = (uint32_t)std::min<uint64_t>(bound_gpk, 128);
        c.sgrid.global_blocks_wide = (uint32_t)std::min<uint64_t>(bound_gwide, 128);
        c.uni_t = uniform_of(pt);
        c.nb_t = pt.back();
        put(c.d_pt, pt);
        c.uni_tc = uniform_of(ptc);
        c.nb_tc = ptc.back();
        put(c.d_ptc, ptc);
        std::vector<uint32_t> pa(1, 0);
        for (auto &w : c.aw) pa.push_back(pa.back() + (uint32_t)p.jobs[(size_t)w.job].N * (uint32_t)w.nslab);
        // the masks of a work are consecutive equal-size pool slices: one
        // stride between their buffers
        for (auto &w : c.aw) {
            const MaskWork *mw = &p.mw[(size_t)w.mfirst];
            w.mstride = w.nmask > 1 ? (int64_t)((const char *)mw[1].info - (const char *)mw[0].info) : 0;
            for (int i = 1; i < w.nmask; ++i)
                if ((const char *)mw[i].info - (const char *)mw[0].info != (int64_t)i * w.mstride ||
                    (const char *)mw[i].E - (const char *)mw[0].E != (int64_t)i * w.mstride) {
                    set_error("internal: the position sets of an accumulation work are not evenly spaced");
                    return GAKCO_EUNSUPPORTED;
                }
        }
        if (c.nacc) memcpy(blob + c.d_acc, c.aw.data(), sizeof(AccWork) * c.aw.size());
        put(c.d_pacc, pa);
        c.nb_acc = pa.back();
    }
    if (!p.mw.empty()) memcpy(blob + p.d_masks, p.mw.data(), sizeof(MaskWork) * p.mw.size());
    put(p.d_pv, pv); put(p.d_px, px); put(p.d_pd, pd); put(p.d_pf, pf);
    put(p.d_pdense, pdn); put(p.d_pdtile, pdt);
    p.nb_v = pv.back(); p.nb_x = px.back(); p.nb_d = pd.back(); p.nb_f = pf.back();
    p.nb_dense = pdn.back(); p.nb_dtile = pdt.back();
    return GAKCO_OK;
}

gakco_status plan_upload(Plan &p, hipStream_t st)
{
    // the blob lives as long as the plan; the call that owns the plan waits
    // for the stream before the plan goes away
    GK_HIP(hipMemcpyAsync(p.base + p.o_desc, p.desc_host.data(), p.desc_bytes, hipMemcpyHostToDevice, st));
    return GAKCO_OK;
}

static const char *kPhaseNames[PH_COUNT] = {"fill", "validate", "extract", "bucket_count", "bucket_scan",
                                            "bucket_scatter", "sort_wave", "sort_wave_big", "sort_block", "sort_global",
                                            "accumulate", "dense_syrk", "dense_clear",
                                            "diag", "finalize", "rows_kdiag", "rows", "rows_finalize",
                                            "direct_count", "direct_excess", "rows_qdiag", "rows_count",
                                            "rows_gemm"};
const char *phase_name(int phase) { return (phase >= 0 && phase < PH_COUNT) ? kPhaseNames[phase] : ""; }

gakco_status prof_begin(gakco_ctx *ctx, hipStream_t st, size_t *slot)
{
    if (!ctx->prof_on) return GAKCO_OK;
    while (ctx->ev_pool.size() < ctx->ev_used + 2) {
        hipEvent_t e;
        GK_HIP(hipEventCreate(&e));
        ctx->ev_pool.push_back(e);
    }
    *slot = ctx->ev_used;
    ctx->ev_used += 2;
    GK_HIP(hipEventRecord(ctx->ev_pool[*slot], st));
    return GAKCO_OK;
}

gakco_status prof_end(gakco_ctx *ctx, hipStream_t st, int phase, size_t slot)
{
    if (!ctx->prof_on) return GAKCO_OK;
    GK_HIP(hipEventRecord(ctx->ev_pool[slot + 1], st));
    ctx->ev_pending.emplace_back(phase, slot);
    return GAKCO_OK;
}

gakco_status prof_collect(gakco_ctx *ctx)
{
    for (auto &pe : ctx->ev_pending) {
        float ms = 0.f;
        GK_HIP(hipEventSynchronize(ctx->ev_pool[pe.second + 1]));
        GK_HIP(hipEventElapsedTime(&ms, ctx->ev_pool[pe.second], ctx->ev_pool[pe.second + 1]));
        ctx->prof_ms[pe.first] += ms;
        ctx->prof_n[pe.first] += 1;
    }
    ctx->ev_pending.clear();
    ctx->ev_used = 0;
    return GAKCO_OK;
}

gakco_status plan_launch(gakco_ctx *ctx, Plan &p, hipStream_t st)
{
    char *d = p.base + p.o_desc;
    const JobDev *jobs = reinterpret_cast<const JobDev *>(d + p.d_jobs);
    const MaskWork *masks = reinterpret_cast<const MaskWork *>(d + p.d_masks);
    auto P = [&](size_t off) { return reinterpret_cast<const uint32_t *>(d + off); };
    const int nj = (int)p.jobs.size();
    // (C_m needs no clearing: the first accumulation work of every level
    // stores its rows)
    GK_PHASE(PH_FILL, launch_fill_u32(reinterpret_cast<uint32_t *>(p.base + p.o_flags), p.nflags, 0u, st));
    GK_PHASE(PH_VALIDATE, launch_validate(jobs, P(p.d_pv), nj, p.nb_v, st));
    GK_PHASE(PH_EXTRACT, launch_extract(jobs, P(p.d_px), nj, p.nb_x, st));
    if (p.n_dwork) {
        const DirectLevel *dlev = reinterpret_cast<const DirectLevel *>(d + p.d_dlev);
        const ExcessList ex{reinterpret_cast<uint4 *>(p.base + p.o_excess),
                            reinterpret_cast<uint32_t *>(p.base + p.o_flags) + p.f_excess, p.excess_cap};
        for (auto &dc : p.dclass)
            GK_PHASE(PH_DIRECT, launch_direct_count(jobs, dlev, reinterpret_cast<const DirectWork *>(d + p.d_dwork),
                                                    reinterpret_cast<const uint2 *>(d + p.d_dchunk) + dc.first,
                                                    P(dc.d_pre), dc.nchunk, dc.uniform, dc.nblocks, dc.kp, ex, st));
        GK_PHASE(PH_DIRECT_EXCESS, launch_direct_excess(jobs, dlev, ex, st));
    }
    if (p.n_dense) ctx->dense_dirty = true;  // the bucket sort writes count rows from here on
    // Independent kernels overlap on the side stream: the block sort beside
    // the wave sort (different buckets), and, after the last chunk's sorts,
    // the int8 products beside the last accumulation (different outputs).
    // Not while profiling (per-kernel times), with the "overlap" parameter
    // 0, or while the stream is being captured into a graph.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    GK_HIP(hipStreamIsCapturing(st, &cap));
    const bool dual = ctx->side && ctx->overlap && !ctx->prof_on && (cap == hipStreamCaptureStatusNone || ctx->capture_side);
    auto fork = [&](int i) -> gakco_status {
        GK_HIP(hipEventRecord(ctx->fork_ev[i], st));
        GK_HIP(hipStreamWaitEvent(ctx->side, ctx->fork_ev[i], 0));
        return GAKCO_OK;
    };
    auto join = [&](int i) -> gakco_status {
        GK_HIP(hipEventRecord(ctx->join_ev[i], ctx->side));
        GK_HIP(hipStreamWaitEvent(st, ctx->join_ev[i], 0));
        return GAKCO_OK;
    };
    // pair updates of the row accumulation (profiling count, spread slots)
    unsigned long long *acc_upd = ctx->prof_on && ctx->prof_stat ? ctx->prof_stat + kProfUpdFirst : nullptr;
    const DenseWork *dw = reinterpret_cast<const DenseWork *>(d + p.d_dense);
    bool dense_done = false;
    size_t ci = 0;
    for (auto &c : p.chunks) {
        const bool last = ++ci == p.chunks.size();
        const MaskWork *cm = masks + c.mfirst;
        uint32_t *bcnt = reinterpret_cast<uint32_t *>(p.base + p.o_pool + c.o_bcnt);
        // one job's diagonal counters, [M+1][N] in one array: summed in LDS if small
        uint32_t *diag0 = nullptr;
        uint32_t ndiag = 0;
        if (p.jobs.size() == 1 && !p.jobs[0].ext_diag.empty()) {
            const size_t nd = (size_t)(p.jobs[0].M + 1) * (size_t)p.jobs[0].N;
            if (nd <= kDiagLds) {
                diag0 = p.jobs[0].ext_diag[0];
                ndiag = (uint32_t)nd;
            }
        }
        const SortLists L{bcnt + c.nbuck, reinterpret_cast<uint32_t *>(p.base + p.o_pool + c.o_lists), (uint32_t)c.nbuck,
                          ctx->prof_on ? ctx->prof_stat : nullptr, diag0, ndiag};
        GK_PHASE(PH_FILL, launch_fill_u32(reinterpret_cast<uint32_t *>(p.base + p.o_pool + c.o_bcnt), c.nbcnt, 0u, st));
        GK_PHASE(PH_BCOUNT, launch_bucket_count(cm, P(c.d_ptc), c.nmask, c.uni_tc, c.nb_tc, c.maxB, st));
        GK_PHASE(PH_BSCAN, launch_bucket_scan(cm, c.nmask, L, st));
        GK_PHASE(PH_BSCATTER, launch_bucket_scatter(cm, P(c.d_pt), c.nmask, c.uni_t, c.nb_t, c.maxB, st));
        if (dual) {
            // the sorts run one after another: each fills the device, and
            // side by side they measured slower than in sequence
            GK_HIP(launch_sort_wave(cm, L, c.sgrid, st));
            GK_HIP(launch_sort_wave_big(cm, L, c.sgrid, st));
            GK_HIP(launch_sort_block(cm, L, c.sgrid, st));
            GK_HIP(launch_sort_global(cm, L, c.sgrid, st));
            if (last && p.n_dense + p.n_dlev) {
                GK_TRY(fork(1));
                GK_HIP(launch_dense_syrk(dw, P(p.d_pdense), p.n_dense + p.n_dlev, p.nb_dense, ctx->side));
                GK_HIP(launch_dense_clear(dw, p.n_dense, ctx->side));
                dense_done = true;
            }
            if (c.nacc)
                GK_HIP(launch_accumulate(jobs, masks, reinterpret_cast<const AccWork *>(d + c.d_acc), P(c.d_pacc), c.nacc,
                                         c.nb_acc, c.acc_lds, acc_upd, st));
            if (dense_done) GK_TRY(join(1));
            continue;
        }
        GK_PHASE(PH_SORT_WAVE, launch_sort_wave(cm, L, c.sgrid, st));
        GK_PHASE(PH_SORT_WAVE_BIG, launch_sort_wave_big(cm, L, c.sgrid, st));
        GK_PHASE(PH_SORT_BLOCK, launch_sort_block(cm, L, c.sgrid, st));
        GK_PHASE(PH_SORT_GLOBAL, launch_sort_global(cm, L, c.sgrid, st));
        if (c.nacc)
            GK_PHASE(PH_ACCUM, launch_accumulate(jobs, masks, reinterpret_cast<const AccWork *>(d + c.d_acc), P(c.d_pacc),
                                                 c.nacc, c.nb_acc, c.acc_lds, acc_upd, st));
    }
    if (p.n_dense + p.n_dlev && !dense_done) {
        GK_PHASE(PH_DENSE_SYRK, launch_dense_syrk(dw, P(p.d_pdense), p.n_dense + p.n_dlev, p.nb_dense, st));
        GK_PHASE(PH_DENSE_CLEAR, launch_dense_clear(dw, p.n_dense, st));
    }
    if (p.n_dense) ctx->dense_dirty = false;
    if (p.nb_d) {
        GK_PHASE(PH_DIAG, launch_diag(jobs, P(p.d_pd), nj, p.nb_d, p.maxM, st));
        GK_PHASE(PH_FINALIZE, launch_finalize(jobs, P(p.d_pf), nj, p.nb_f, p.maxM, st));
    }
    ctx->last_chunks = (int64_t)p.chunks.size();
    return GAKCO_OK;
}

gakco_status plan_check_errors(gakco_ctx *ctx, Plan &p, hipStream_t st)
{
    std::vector<int32_t> flags(p.nflags, 0);
    GK_HIP(hipMemcpyAsync(flags.data(), p.base + p.o_flags, flags.size() * 4, hipMemcpyDeviceToHost, st));
    GK_HIP(hipStreamSynchronize(st));
    GK_TRY(prof_collect(ctx));
    ctx->last_dense_rows = 0;
    for (size_t i = p.jobs.size(); i < p.f_excess; ++i) ctx->last_dense_rows += (uint32_t)flags[i];
    ctx->last_excess = (uint32_t)flags[p.f_excess];
    ctx->last_direct_levels = p.n_dlev;
    gakco_status first = GAKCO_OK;
    for (size_t j = 0; j < p.jobs.size(); ++j) {
        if (flags[j] & 2) {
            p.excess_overflow = true;
            p.jobs[j].status = GAKCO_EUNSUPPORTED;
            if (first == GAKCO_OK) {
                set_error("job %zu: more than %u counts above 127 in directly addressed position sets", j, p.excess_cap);
                first = GAKCO_EUNSUPPORTED;
            }
        } else if (flags[j] & 1) {
            p.jobs[j].status = GAKCO_ERANGE;
            if (first == GAKCO_OK) {
                set_error("job %zu: a symbol code lies outside [0, sigma=%d)", j, p.jobs[j].sigma);
                first = GAKCO_ERANGE;
            }
        } else {
            p.jobs[j].status = GAKCO_OK;
        }
    }
    return first;
}

}  // namespace gk
