// Direct-address grouping (no sort) of levels with a small reduced-g-mer
// space: count-matrix rows written straight from per-sequence histograms,
// and the exact correction of counts above 127.
//
// For a position set of level m, two g-mers are in one group of Algorithm 1
// exactly when their reduced (g-m)-mers are equal, so the group of a reduced
// g-mer u is the row "u" of a count matrix D with D[X][u] = the number of
// g-mers of sequence X whose reduced form is u.  The group's contribution
// count_X * count_Y to C_m[X][Y] (countAndUpdate) summed over all groups and
// all position sets of the level is (D^T D)[X][Y], which the int8 matrix-core
// kernel computes from the rows written here.
#include "common.h"
#include "launch.h"

namespace gk {

// Row of reduced g-mer rk inside its position set: the compacted key itself
// when sigma is a power of two, else its base-sigma value.
__device__ __forceinline__ uint32_t direct_row(uint64_t rk, const DirectLevel &L)
{
    if (L.pow2) return (uint32_t)rk;
    const uint64_t fm = bits_mask(L.b);
    uint32_t v = 0;
    for (int d = L.nd - 1; d >= 0; --d) v = v * (uint32_t)L.sigma + (uint32_t)((rk >> (d * L.b)) & fm);
    return v;
}

// One block per (chunk of position sets of one level, sequence X < Ntile):
// for each position set of the chunk, an LDS histogram of X's reduced
// g-mers, then the Kp bytes of X's row segment written as 16-byte stores
// (counts clipped at 127, the excess appended to the list).
// Blocks of padding sequences (X >= N) write zeros; the level's last
// position set also zeroes the row tail [R, stride); its first position set
// clears X's upper row of C_m, to which only the excess corrections add.
__global__ __launch_bounds__(kThreads) void k_direct_count(const JobDev *__restrict__ jobs,
                                                           const DirectLevel *__restrict__ dlev,
                                                           const DirectWork *__restrict__ dwork,
                                                           const uint2 *__restrict__ chunks,
                                                           const uint32_t *__restrict__ bprefix, int nchunk,
                                                           uint32_t uniform, ExcessList ex)
{
    extern __shared__ uint32_t hist[];
    int ci;
    uint32_t X;
    map_block(bprefix, nchunk, uniform, blockIdx.x, ci, X);
    const uint2 ch = chunks[ci];
    const DirectLevel &L = dlev[dwork[ch.x].dl];
    const JobDev &J = jobs[L.job];
    const uint32_t N = (uint32_t)J.N, Kp = L.Kp;
    const int tid = threadIdx.x;
    const uint32_t t0 = X < N ? J.gstart[X] : 0u, t1 = X < N ? J.gstart[X + 1] : 0u;
    const gptr<const uint64_t> key = glb((const uint64_t *)J.key);
#pragma unroll 1
    for (uint32_t k = 0; k < ch.y; ++k) {
        const DirectWork &W = dwork[ch.x + k];
        for (uint32_t i = tid; i < Kp; i += kThreads) hist[i] = 0;
        __syncthreads();
        if (W.first && X < N) {
            const gptr<int64_t> crow = glb(J.C) + ((size_t)L.level * N + X) * (size_t)N;
            for (uint32_t Y = X + tid; Y < N; Y += kThreads) crow[Y] = 0;
        }
        for (uint32_t t = t0 + tid; t < t1; t += kThreads) {
            // rows past Kp come only from symbols outside [0, sigma), which
            // fail the call; they are dropped here
            const uint32_t r = direct_row(compact_key(key[t], W.md), L);
            if (r < Kp) atomicAdd(&hist[r], 1u);
        }
        __syncthreads();
        // X's row segment [row0, row0 + n): 16-byte pieces of the tiled layout
        // (row0 and Kp are multiples of 16)
        const gptr<int8_t> D = glb(L.D);
        const uint32_t n = Kp + (W.last ? L.stride - L.R : 0u);
        for (uint32_t i = (uint32_t)tid * 16u; i < n; i += kThreads * 16u) {
            uint32_t wv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t v = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const uint32_t r = i + (uint32_t)(q * 4 + b);
                    uint32_t c = r < Kp ? hist[r] : 0u;
                    if (c > 127u) {
                        const uint32_t e = g_atomic_add(glb(ex.count), 1u);
                        if (e < ex.cap) st_u4(glb(ex.ent), e, W.row0 + r, X, c - 127u, (uint32_t)W.dl);
                        else atomicOr(J.err, 2);
                        c = 127u;
                    }
                    v |= c << (8 * b);
                }
                wv[q] = v;
            }
            *(gptr<u32x4>)(D + tiled_offset(X, (size_t)W.row0 + i, L.stride)) = u32x4{wv[0], wv[1], wv[2], wv[3]};
        }
        __syncthreads();
    }
}

// Exact correction for clipped counts.  With a = min(c, 127) and e = c - a,
// a row's product c_X c_Y for a pair X != Y exceeds what D holds, a_X a_Y, by
// e_X a_Y + a_X e_Y + e_X e_Y, and the diagonal's c_Z^2 exceeds a_Z^2 by
// 2 a_Z e_Z + e_Z^2.  One block per excess entry (r, Z, e_Z) adds e_Z a_W to
// the pair (Z, W) for every other sequence W of the row (read from D's
// column r), the diagonal term to (Z, Z), and e_Z e_W for every later entry
// (r, W, e_W) of the same row (the list is short: a pairwise scan).
// Global 64-bit atomics into the level's C_m, upper triangle.
__global__ __launch_bounds__(kThreads) void k_direct_excess(const JobDev *__restrict__ jobs,
                                                            const DirectLevel *__restrict__ dlev, ExcessList ex)
{
    const uint32_t n = min(*(volatile uint32_t *)ex.count, ex.cap);
    const gptr<const u32x4> ent = (gptr<const u32x4>)glb((const uint4 *)ex.ent);
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
        const u32x4 e = ent[i];
        const DirectLevel &L = dlev[e.w];
        const JobDev &J = jobs[L.job];
        const uint32_t N = (uint32_t)J.N, r = e.x, Z = e.y;
        const uint64_t eZ = e.z;
        const gptr<uint64_t> C = glb(reinterpret_cast<uint64_t *>(J.C)) + (size_t)L.level * N * N;
        const gptr<const uint8_t> D = glb((const uint8_t *)L.D);
        for (uint32_t Y = threadIdx.x; Y < N; Y += kThreads) {
            if (Y == Z) {
                g_atomic_add(C + (size_t)Z * N + Z, eZ * (2u * 127u + eZ));
                continue;
            }
            const uint64_t a = D[tiled_offset(Y, r, L.stride)];
            if (a) g_atomic_add(C + (size_t)min(Y, Z) * N + max(Y, Z), a * eZ);
        }
        for (uint32_t j = i + 1 + threadIdx.x; j < n; j += kThreads) {
            const u32x4 f = ent[j];
            if (f.x == r && f.w == e.w)
                g_atomic_add(C + (size_t)min(Z, f.y) * N + max(Z, f.y), eZ * (uint64_t)f.z);
        }
    }
}

hipError_t launch_direct_count(const JobDev *jobs, const DirectLevel *dlev, const DirectWork *dwork, const uint2 *chunks,
                               const uint32_t *bprefix, int nchunk, uint32_t uniform, uint32_t nblocks, uint32_t maxKp,
                               ExcessList ex, hipStream_t st)
{
    if (!nblocks) return hipSuccess;
    hipLaunchKernelGGL(k_direct_count, dim3(nblocks), dim3(kThreads), (size_t)maxKp * 4, st, jobs, dlev, dwork, chunks,
                       bprefix, nchunk, uniform, ex);
    return hipGetLastError();
}

hipError_t launch_direct_excess(const JobDev *jobs, const DirectLevel *dlev, ExcessList ex, hipStream_t st)
{
    hipLaunchKernelGGL(k_direct_excess, dim3(256), dim3(kThreads), 0, st, jobs, dlev, ex);
    return hipGetLastError();
}

}  // namespace gk
