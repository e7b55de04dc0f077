// Host-side launchers of the gfx950 kernels (one per kernel family).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gk {
struct MaskDesc;
struct JobDev;
struct MaskWork;
struct AccWork;
struct DenseWork;
struct RowsWork;
struct DirectLevel;
struct DirectWork;
struct ExcessList;

hipError_t launch_fill_u64(uint64_t *p, size_t n, uint64_t v, hipStream_t st);
hipError_t launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t st);
hipError_t launch_validate(const JobDev *jobs, const uint32_t *bprefix, int njobs, uint32_t nblocks, hipStream_t st);
hipError_t launch_extract(const JobDev *jobs, const uint32_t *bprefix, int njobs, uint32_t nblocks, hipStream_t st);
hipError_t launch_bucket_count(const MaskWork *items, const uint32_t *bprefix, int nitems, uint32_t uniform, uint32_t nblocks,
                               int maxB, hipStream_t st);
struct SortLists;
// Grid sizes of the per-bucket sort kernels (0 = not launched).
struct SortGrid {
    uint32_t wave_blocks = 0, wave_big_blocks = 0, block_blocks = 0, global_blocks_pk = 0, global_blocks_wide = 0;
};
hipError_t launch_bucket_scan(const MaskWork *items, int nitems, SortLists L, hipStream_t st);
hipError_t launch_bucket_scatter(const MaskWork *items, const uint32_t *bprefix, int nitems, uint32_t uniform, uint32_t nblocks,
                                 int maxB, hipStream_t st);
hipError_t launch_sort_wave(const MaskWork *items, SortLists L, const SortGrid &g, hipStream_t st);
hipError_t launch_sort_wave_big(const MaskWork *items, SortLists L, const SortGrid &g, hipStream_t st);
hipError_t launch_sort_block(const MaskWork *items, SortLists L, const SortGrid &g, hipStream_t st);
hipError_t launch_sort_global(const MaskWork *items, SortLists L, const SortGrid &g, hipStream_t st);
hipError_t launch_accumulate(const JobDev *jobs, const MaskWork *items, const AccWork *aw, const uint32_t *bprefix, int nacc,
                             uint32_t nblocks, size_t lds_bytes, unsigned long long *updates, hipStream_t st);
// Random-address LDS atomic adds over a row of row_words (a power of two)
// counters, as the row accumulation issues them: updates per second.
hipError_t probe_lds_atomics(int row_words, double *updates_per_s);
hipError_t launch_diag(const JobDev *jobs, const uint32_t *bprefix, int njobs, uint32_t nblocks, int maxM, hipStream_t st);
hipError_t launch_dense_syrk(const DenseWork *dw, const uint32_t *bprefix, int nwork, uint32_t nblocks, hipStream_t st);
hipError_t launch_dense_clear(const DenseWork *dw, int nwork, hipStream_t st);
size_t dense_work_size();
int dense_tile();
int dense_kchunk();
uint32_t dense_split_rows();
void dense_work_fill(void *dst, int8_t *Dt, const uint32_t *count, uint32_t cap, uint32_t stride, int N, int nt, int S,
                     int32_t *P);
size_t res_mask_size();
void res_mask_fill(void *dst, const MaskDesc &md, int w, int B, int hb, int sb, const uint32_t *boff, const uint32_t *bgrp,
                   const uint32_t *E, const uint4 *gtab);
hipError_t launch_query_diag(const uint64_t *qkey, const uint32_t *qgstart, int nq, int nmask, int tbits, const void *rm,
                             uint32_t *diag, hipStream_t st);
hipError_t launch_count_rows(const uint64_t *key, const uint32_t *gstart, int nseq, const void *rm, int nset, int w,
                             int8_t *out, size_t stride, uint32_t *flag, hipStream_t st);
// S column splits (S <= 0: chosen from the device's resident blocks)
hipError_t launch_rows_gemm(const int8_t *Q, const int8_t *D, size_t stride, int nq, int nsv, int S, const uint32_t *qflag,
                            uint32_t *C, hipStream_t st);
int rows_gemm_tile_q(int nq);
int rows_gemm_tile_sv();
hipError_t launch_rows(const uint64_t *qkey, const uint32_t *qgstart, int nq, int M, int nsv, int slab, int mchunk,
                       int nitems, const void *rm, const int32_t *lev_first, const int32_t *lev_count, uint32_t *C,
                       unsigned long long *updates, int dense_level, const uint32_t *qflag, hipStream_t st);
hipError_t launch_kdiag_counts(const uint32_t *diag, int n, int M, const int64_t *coef, const int64_t *hco, int64_t *Kd,
                               hipStream_t st);
hipError_t launch_rows_finalize(const uint32_t *C, int nq, int nsv, int M, const int64_t *coef, const int64_t *hco,
                                const int64_t *Kd_sv, const int64_t *Kd_q, const double *alpha, double bias, double *K_rows,
                                int64_t ldk, int64_t *Nm_rows, double *decision, double *partial, hipStream_t st);
hipError_t launch_mirror_block(double *out, int64_t ld, int rows, int c0, int cols, hipStream_t st);
size_t rows_partial_count(int nq, int nsv);
hipError_t init_rows_attributes(size_t lds);
hipError_t launch_direct_count(const JobDev *jobs, const DirectLevel *dlev, const DirectWork *dwork, const uint2 *chunks,
                               const uint32_t *bprefix, int nchunk, uint32_t uniform, uint32_t nblocks, uint32_t maxKp,
                               ExcessList ex, hipStream_t st);
hipError_t launch_direct_excess(const JobDev *jobs, const DirectLevel *dlev, ExcessList ex, hipStream_t st);
hipError_t launch_finalize(const JobDev *jobs, const uint32_t *bprefix, int njobs, uint32_t nblocks, int maxM, hipStream_t st);
}  // namespace gk
