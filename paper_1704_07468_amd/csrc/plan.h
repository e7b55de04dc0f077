// Host-side planning of Gram jobs: validation, g-mer offsets, position sets,
// bucket geometry, device memory layout and the launch sequence.  Shared by
// the single-job path, the batched path and the resident-set builder.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/gakco.h"
#include "common.h"
#include "launch.h"

// Phases timed by the optional event profiler (hipEvents around launches).
// Each phase is one kernel launch (or none) per chunk of a call.
enum GkPhase { PH_FILL, PH_VALIDATE, PH_EXTRACT, PH_BCOUNT, PH_BSCAN, PH_BSCATTER, PH_SORT_WAVE, PH_SORT_WAVE_BIG, PH_SORT_BLOCK,
               PH_SORT_GLOBAL, PH_ACCUM, PH_DENSE_SYRK, PH_DENSE_CLEAR, PH_DIAG, PH_FINALIZE,
               PH_ROWS_KDIAG, PH_ROWS, PH_ROWS_FINALIZE, PH_DIRECT, PH_DIRECT_EXCESS, PH_ROWS_QDIAG,
               PH_ROWS_COUNT, PH_ROWS_GEMM, PH_COUNT };

// profiling counter slots: six sort kinds, then the row accumulation's pair
// updates spread over kProfUpdSlots slots (one per block residue) so that the
// counting adds no same-address contention to the timed kernel
constexpr int kProfUpdFirst = 8, kProfUpdSlots = 256;
constexpr int kProfRowsFirst = kProfUpdFirst + kProfUpdSlots;  // then the serving rows' pair updates
constexpr int kProfStatSlots = kProfRowsFirst + kProfUpdSlots;
// entries of the clipped-count list of one call (a pairwise scan corrects them)
constexpr uint32_t kExcessCap = 262144;

struct gakco_ctx {
    int device = 0;
    size_t budget = 0;
    int dense_tau = 0;       // 0 = int8 matrix-core path off
    int bucket_avg = 512;    // target g-mers per hash bucket
    int acc_slab = 0;        // columns per row-accumulation block (0: as many as the LDS holds)
    int acc_mstep = 0;       // cap on position sets per flush of the row accumulation (0: the count bound only)
    int rows_slabs = 0;      // resident slabs of the serving rows kernel (0: halves of 4096..16384 sequences)
    int rows_dense = 1;      // 1: join the resident set's top level on the matrix cores when it qualifies
    int rows_dense_min_sv = 2048;  // ... for resident sets of at least this many sequences
    int rows_dense_min_q = 28;     // ... and query batches of at least this many queries
    int direct_mode = 1;     // direct-address levels: 0 off, 1 where the cost model prefers them, 2 wherever possible
    uint32_t excess_cap = 0; // cap on the clipped-count list (0: kExcessCap), for tests
    int chunk_masks = 0;     // cap on position sets per chunk (0: as many as the pool holds)
    int info4 = 1;           // 4-byte per-g-mer run records where they fit (0: uint2 records)
    size_t pool_cap = 16ull << 30;  // per-chunk partition/sort buffers
    void *arena = nullptr;
    size_t arena_cap = 0;
    size_t lds_max = 0;      // dynamic LDS available to the row accumulation
    // count matrices of the int8 matrix-core path: kept all-zero between
    // calls (each call clears the rows it used)
    int8_t *dense_buf = nullptr;
    size_t dense_cap = 0;
    bool dense_dirty = false;
    // event profiler
    bool prof_on = false;
    unsigned long long *prof_stat = nullptr;  // device, profiling only: g-mers per sort kind, pair updates
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, size_t>> ev_pending;  // (phase, first of two events)
    double prof_ms[PH_COUNT] = {};
    int64_t prof_n[PH_COUNT] = {};
    // autotuned int8 path threshold per job class (symbol bits * 100 + g)
    std::map<int, int> class_tau;
    // second stream (default priority) and fork/join events: the block sort
    // runs beside the wave sort, the int8 products beside the accumulation
    hipStream_t side = nullptr;
    bool overlap = true;
    bool capture_side = false;  // the side stream also joins a graph capture (batch plans)
    hipEvent_t fork_ev[2] = {nullptr, nullptr}, join_ev[2] = {nullptr, nullptr};
    // statistics of the last call
    int64_t last_dense_rows = 0;
    int64_t last_chunks = 0;
    int64_t last_excess = 0;  // counts above 127 in directly addressed position sets
    int64_t last_direct_levels = 0;  // levels grouped by direct addressing
    int64_t direct_fallbacks = 0;    // calls redone without direct addressing (list overflow)
    // fixed scratch (the allocation-free entry point): arena and count
    // matrices share one caller-given region of arena_cap bytes, nothing is
    // allocated or freed, and the caller's outputs do not count against the
    // budget
    bool fixed_arena = false;
    // a small device buffer (4 KB) for per-call results of the training
    // consumer, allocated on first use
    void *small = nullptr;
};

namespace gk {

void set_error(const char *fmt, ...);
const char *hip_name(hipError_t e);

#define GK_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t _e = (call);                                                        \
        if (_e != hipSuccess) {                                                        \
            ::gk::set_error("%s failed: %s (%s:%d)", #call, ::gk::hip_name(_e), __FILE__, \
                            __LINE__);                                                 \
            return GAKCO_EHIP;                                                         \
        }                                                                              \
    } while (0)

#define GK_TRY(expr)                  \
    do {                              \
        gakco_status _s = (expr);     \
        if (_s != GAKCO_OK) return _s; \
    } while (0)

int64_t binom64(int n, int r);
int symbol_bits(int sigma);

// Bump layout over one device allocation: offsets first, pointers after the
// arena is sized.
struct Layout {
    size_t size = 0;
    size_t take(size_t bytes, size_t align = 256)
    {
        size = (size + align - 1) / align * align;
        size_t off = size;
        size += bytes;
        return off;
    }
};

struct JobPlan {
    // request
    const int8_t *seqs = nullptr;
    const int32_t *lens_dev = nullptr;
    int32_t N = 0, sigma = 0, g = 0, k = 0;
    double *K_out = nullptr;
    int64_t *Nm_out = nullptr;
    int64_t *Cm_out = nullptr;
    bool want_kernel = true;  // run accumulation + epilogue (false: partition only)
    int tau = -1;             // per-job int8 path threshold (-1: the context's)
    // host-side shape
    std::vector<int32_t> lens;
    int M = 0, b = 0, sb = 0;
    uint32_t T = 0, maxng = 0;
    int64_t nsym = 0;
    std::vector<uint32_t> gstart;
    std::vector<int64_t> seq_off;
    std::vector<MaskDesc> masks;
    std::vector<int> level_B;  // bucket bits per level
    // direct-address levels (no sort): their position sets, and per level the
    // count-matrix geometry (0 where the level is sorted)
    std::vector<MaskDesc> dmasks;
    std::vector<char> direct;
    std::vector<uint32_t> dKp, dR, dstride;
    std::vector<int> dSd;           // row splits of its int8 products
    std::vector<size_t> o_Dd, o_Pd; // arena offsets: count matrix, partial tiles
    // layout offsets (arena)
    size_t o_seqoff = 0, o_gstart = 0, o_key = 0, o_sid = 0, o_C = 0, o_Kd = 0, o_coef = 0, o_hco = 0, o_dref = 0;
    std::vector<uint32_t> dcap;  // per level dense row capacity (0 = level has no dense path)
    std::vector<size_t> o_dense; // per level offset in the context's dense buffer
    std::vector<size_t> o_P;     // per level partial tiles of the split rows
    int dS = 1;                  // row splits per dense output tile
    int Npad = 0;                // N rounded up to 64
    int acc_slab = 0, acc_nslab = 1;  // row-accumulation columns per block, blocks per row
    int Ntile = 0;               // sequences padded to the dense tile edge
    bool own_C = false;
    uint64_t *key_override = nullptr;  // write g-mers to caller buffers (stage entry point)
    uint32_t *sid_override = nullptr;
    // serving: caller-owned per-mask tables that outlive the call (bucket
    // offsets, groups per bucket, run entries, group tables) and per-level
    // diagonal counters (zeroed by the caller)
    std::vector<uint32_t *> ext_boff, ext_bgrp, ext_E;
    std::vector<uint4 *> ext_gtab;
    std::vector<uint32_t *> ext_diag;
    // device view
    JobDev dev{};
    int mask_first = 0;  // index of its first mask in Plan::mw
    size_t lev_base = 0; // index of its first dense row counter
    int status = GAKCO_OK;
};

// A run of consecutive masks whose partition/sort buffers share the pool.
struct Chunk {
    int mfirst = 0, nmask = 0;
    std::vector<size_t> o_mask;  // pool offset of each mask's buffers
    size_t o_bcnt = 0, nbcnt = 0;  // bucket counts of every mask, then the sort counters
    size_t nbuck = 0;              // buckets of all masks
    size_t o_lists = 0;            // sort class lists, nbuck entries per class
    int maxB = 0;
    SortGrid sgrid;
    // descriptor blob offsets
    size_t d_pt = 0, d_ptc = 0, d_acc = 0, d_pacc = 0;
    uint32_t nb_t = 0, uni_t = 0, nb_tc = 0, uni_tc = 0, nb_acc = 0;  // scatter / count tile grids
    int nacc = 0;
    size_t acc_lds = 0;
    std::vector<AccWork> aw;
};

// The whole plan of one call (one or more jobs).
struct Plan {
    std::vector<JobPlan> jobs;
    std::vector<Chunk> chunks;
    Layout lay;
    size_t o_desc = 0, desc_bytes = 0;
    size_t o_flags = 0;  // per-job error flags, then the dense row counters
    size_t nflags = 0;
    size_t o_pool = 0, pool_bytes = 0;
    std::vector<char> desc_host;  // staged descriptor blob
    size_t d_jobs = 0, d_masks = 0, d_dense = 0, d_pdense = 0, d_pdtile = 0;
    size_t d_pv = 0, d_px = 0, d_pd = 0, d_pf = 0;
    uint32_t nb_v = 0, nb_x = 0, nb_d = 0, nb_f = 0, nb_dense = 0, nb_dtile = 0;
    int n_dense = 0, maxM = 0;
    // direct-address levels of all jobs: level table, one work per position
    // set (blocks: Ntile per work), the row counts their int8 products read,
    // the excess list and its counter (the last flag word)
    int n_dlev = 0, n_dwork = 0, n_dchunk = 0;
    size_t d_dlev = 0, d_dwork = 0, d_dchunk = 0, d_pdir = 0, d_drows = 0;
    // the row writer's launches: chunks of position sets grouped by rows per
    // position set (LDS counters), largest first
    struct DirClass {
        int first = 0, nchunk = 0;
        size_t d_pre = 0;
        uint32_t nblocks = 0, uniform = 0, kp = 0;
    };
    std::vector<DirClass> dclass;
    size_t o_excess = 0, f_excess = 0;
    uint32_t excess_cap = 0;
    bool excess_overflow = false;  // set by plan_check_errors: redo without direct addressing
    size_t dense_bytes = 0, output_bytes = 0;
    std::vector<MaskWork> mw;
    char *base = nullptr;  // arena base
};

gakco_status ctx_small_buffer(gakco_ctx *ctx, void **out);
// Optional ordering of one rows call's device work among others: enter()
// before its first kernel is queued, leave() once all of its kernels are.
struct RowsGate {
    void (*enter)(void *arg, hipStream_t st);
    void (*leave)(void *arg, hipStream_t st);
    void *arg;
};
// Kernel rows of queries against a resident set (serving join); K_rows row
// stride ldk (0: the resident set's size).
gakco_status rows_run(gakco_ctx *ctx, const gakco_resident *R, const int8_t *q_seqs, const int32_t *q_lens,
                      const int32_t *q_lens_host, int32_t n_q, double *K_rows, int64_t ldk, int64_t *Nm_rows,
                      double *decision, hipStream_t st, const RowsGate *gate = nullptr);
gakco_status plan_shape(gakco_ctx *ctx, JobPlan &jp, const int32_t *removed_one, int m_one);
gakco_status plan_layout(gakco_ctx *ctx, Plan &p);
gakco_status plan_bind(gakco_ctx *ctx, Plan &p, hipStream_t st);  // arena + pointers + descriptor blob
gakco_status plan_upload(Plan &p, hipStream_t st);
gakco_status plan_launch(gakco_ctx *ctx, Plan &p, hipStream_t st);
gakco_status fetch_lens(JobPlan &jp, hipStream_t st);
gakco_status plan_check_errors(gakco_ctx *ctx, Plan &p, hipStream_t st);
gakco_status run_single(gakco_ctx *ctx, Plan &p, hipStream_t st);

// Event profiler: prof_begin/prof_end bracket one phase on a stream (no-ops
// unless the context's profiler is on); prof_collect adds the elapsed times
// of completed brackets after the stream has been synchronised.
gakco_status prof_begin(gakco_ctx *ctx, hipStream_t st, size_t *slot);
gakco_status prof_end(gakco_ctx *ctx, hipStream_t st, int phase, size_t slot);
gakco_status prof_collect(gakco_ctx *ctx);
const char *phase_name(int phase);

// Runs `launch` between two profiler events of phase `ph`.
#define GK_PHASE(ph, launch)                         \
    do {                                             \
        size_t _slot = 0;                            \
        GK_TRY(prof_begin(ctx, st, &_slot));         \
        GK_HIP(launch);                              \
        GK_TRY(prof_end(ctx, st, (ph), _slot));      \
    } while (0)

}  // namespace gk
