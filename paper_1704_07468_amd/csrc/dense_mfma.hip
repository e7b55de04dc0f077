// int8 matrix-core path of the count update (Algorithm 1 countAndUpdate) for
// groups with many distinct sequences.
//
// Each such group of a level m is one row r of a count matrix D_m (row r,
// column X = how often sequence X holds the group's reduced g-mer), so the
// group's contribution to C_m is the outer product of that row with itself
// and the contribution of all of them is D_m^T D_m.  Counts are <= 127, so
// int8 operands with int32 accumulation are exact for up to
// 2^31 / 127^2 = 133144 rows; each split of at most 65536 rows keeps its
// exact int32 partial tile, and the epilogue adds the splits into C_m.  D is
// stored sequence-major in tiles of 128 sequences (tiled_offset): a step's
// operand slab of a tile is one contiguous 8 KB block, and every MFMA
// operand is 16 contiguous bytes along r.  Only tiles on or above the diagonal are
// computed; the epilogue mirrors the upper triangle.
#include "common.h"
#include "launch.h"

namespace gk {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kDTile = kDenseTile;    // output tile edge
constexpr int kDK = kDenseK;          // rows (k) staged per LDS buffer
constexpr int kDRow = kDK + 16;       // padded LDS row: 80 bytes keeps 16-byte reads conflict-free
constexpr uint32_t kDSplitRows = kDenseSplitRows;

struct DenseWork {
    int8_t *Dt;              // [Npad][stride] counts (tiled_offset layout), zero beyond the used rows
    const uint32_t *count;   // rows used (device counter)
    uint32_t cap;            // row capacity (<= S * kDSplitRows)
    uint32_t stride;         // bytes per sequence (multiple of kDK, >= cap)
    int32_t N, nt, S;        // sequences, tiles per edge, row splits
    int32_t *P;              // partial tiles [nt*(nt+1)/2][S][128*128]
};

__device__ __forceinline__ void tile_of(int f, int nt, int &I, int &J)
{
    I = 0;
    while (f >= nt - I) {
        f -= nt - I;
        ++I;
    }
    J = I + f;
}

// v_mfma_i32_32x32x32_i8 operand layout: lane l supplies row/column (l % 32)
// and 16 consecutive k values starting at 16*(l/32); accumulator v of lane l
// is element (8*(v/4) + 4*(l/32) + v%4, l % 32).
// One block = one 128x128 upper tile x one split of the rows.  The A (rows
// of the tile) and B (columns) operand slabs of 64 rows are staged through
// double-buffered LDS with coalesced 16-byte loads; each wave computes a
// 64x64 quarter as 2x2 MFMA tiles.  The exact int32 partial tile is stored
// for the epilogue, which adds the splits into C_m.
__global__ __launch_bounds__(kThreads) void k_dense_syrk(const DenseWork *__restrict__ dw, const uint32_t *__restrict__ bprefix,
                                                         int nwork)
{
    __shared__ __attribute__((aligned(16))) int8_t sA[2][kDTile][kDRow];
    __shared__ __attribute__((aligned(16))) int8_t sB[2][kDTile][kDRow];
    const int wi = find_item(bprefix, nwork, blockIdx.x);
    const DenseWork &W = dw[wi];
    const uint32_t R = min(*W.count, W.cap);
    const int flat = (int)(blockIdx.x - bprefix[wi]);
    const int f = flat / W.S, sp = flat - f * W.S;
    uint32_t r0, r1;
    split_range(R, W.S, sp, r0, r1);
    if (r0 >= r1) return;
    int I, J;
    tile_of(f, W.nt, I, J);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wx = wave & 1, wy = wave >> 1;
    // staging: thread -> (row, 16-byte column) pairs of the 128 x 64 slabs
    const int lr = tid >> 2, lc = (tid & 3) * 16;  // rows lr and lr + 64
    // tiled layout: sequence tile I, 64-row step r at I 128 stride + 128 r,
    // sequence lr + 64 j of the tile 64 (lr + 64 j) further
    const gptr<const int8_t> ga = glb((const int8_t *)W.Dt) + (size_t)I * kDTile * W.stride + lr * 64 + lc;
    const gptr<const int8_t> gb = glb((const int8_t *)W.Dt) + (size_t)J * kDTile * W.stride + lr * 64 + lc;
    // operand slabs of one 64-row step, in registers on their way to LDS
    struct Slab {
        v4i a0, a1, b0, b1;
    };
    auto gload = [&](uint32_t r, Slab &x) {
        const size_t o = (size_t)r * 128u;  // r is a multiple of 64
        x.a0 = *(gptr<const v4i>)(ga + o);
        x.a1 = *(gptr<const v4i>)(ga + 4096 + o);
        x.b0 = *(gptr<const v4i>)(gb + o);
        x.b1 = *(gptr<const v4i>)(gb + 4096 + o);
    };
    auto lstore = [&](int buf, const Slab &x) {
        *reinterpret_cast<v4i *>(&sA[buf][lr][lc]) = x.a0;
        *reinterpret_cast<v4i *>(&sA[buf][lr + 64][lc]) = x.a1;
        *reinterpret_cast<v4i *>(&sB[buf][lr][lc]) = x.b0;
        *reinterpret_cast<v4i *>(&sB[buf][lr + 64][lc]) = x.b1;
    };
    v16i acc00 = {}, acc01 = {}, acc10 = {}, acc11 = {};
    const int fr = lane & 31, fk = 16 * (lane >> 5);
    auto compute = [&](int buf) {
#pragma unroll
        for (int kk = 0; kk < kDK; kk += 32) {
            const v4i a0 = *reinterpret_cast<const v4i *>(&sA[buf][wx * 64 + fr][kk + fk]);
            const v4i a1 = *reinterpret_cast<const v4i *>(&sA[buf][wx * 64 + 32 + fr][kk + fk]);
            const v4i b0 = *reinterpret_cast<const v4i *>(&sB[buf][wy * 64 + fr][kk + fk]);
            const v4i b1 = *reinterpret_cast<const v4i *>(&sB[buf][wy * 64 + 32 + fr][kk + fk]);
            acc00 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, b0, acc00, 0, 0, 0);
            acc01 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, b1, acc01, 0, 0, 0);
            acc10 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, b0, acc10, 0, 0, 0);
            acc11 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, b1, acc11, 0, 0, 0);
        }
    };
    // Two steps of loads in flight: while step r is multiplied from LDS, the
    // slabs of step r + 64 (already loaded) go to the other buffer and those
    // of step r + 128 are loaded.  Loads past the split's last step re-read
    // that step (rows up to a multiple of 64 past the used rows are zero and
    // allocated), so no load is conditional.
    const uint32_t last = r0 + (r1 - r0 - 1) / kDK * kDK;
    Slab x0, x1;
    gload(r0, x0);
    gload(min(r0 + kDK, last), x1);
    lstore(0, x0);
    __syncthreads();
    auto step = [&](uint32_t r, int buf, Slab &ld, const Slab &st) {
        gload(min(r + 2 * kDK, last), ld);
        compute(buf);
        lstore(buf ^ 1, st);
        __syncthreads();
    };
    uint32_t r = r0;
#pragma unroll 1
    while (true) {
        step(r, 0, x0, x1);  // x1: step r + 64; x0 <- step r + 128
        r += kDK;
        if (r >= r1) break;
        step(r, 1, x1, x0);
        r += kDK;
        if (r >= r1) break;
    }
    const gptr<int32_t> P = glb(W.P) + ((size_t)f * W.S + sp) * (kDTile * kDTile);
    auto put = [&](const v16i &acc, int xb, int yb) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int xl = xb + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
            P[dense_tile_offset(xl, yb + (lane & 31))] = acc[v];
        }
    };
    put(acc00, wx * 64, wy * 64);
    put(acc01, wx * 64, wy * 64 + 32);
    put(acc10, wx * 64 + 32, wy * 64);
    put(acc11, wx * 64 + 32, wy * 64 + 32);
}

// Restore the zero invariant of Dt: clear the used rows of every sequence.
__global__ __launch_bounds__(kThreads) void k_dense_clear(const DenseWork *__restrict__ dw, int nwork)
{
    const DenseWork &W = dw[blockIdx.y];
    const uint32_t R = min(*W.count, W.cap);
    const uint32_t nv = (R + 15) / 16;  // 16-byte words per sequence row (stride is a multiple of 64)
    const size_t total = (size_t)W.N * nv;
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < total; i += (size_t)gridDim.x * kThreads) {
        const size_t x = i / nv, q = i - x * nv;
        *(gptr<v4i>)(glb(W.Dt) + tiled_offset((uint32_t)x, q * 16, W.stride)) = v4i{0, 0, 0, 0};
    }
    (void)nwork;
}

hipError_t launch_dense_syrk(const DenseWork *dw, const uint32_t *bprefix, int nwork, uint32_t nblocks, hipStream_t st)
{
    if (!nblocks) return hipSuccess;
    hipLaunchKernelGGL(k_dense_syrk, dim3(nblocks), dim3(kThreads), 0, st, dw, bprefix, nwork);
    return hipGetLastError();
}



hipError_t launch_dense_clear(const DenseWork *dw, int nwork, hipStream_t st)
{
    if (!nwork) return hipSuccess;
    hipLaunchKernelGGL(k_dense_clear, dim3(1024, nwork), dim3(kThreads), 0, st, dw, nwork);
    return hipGetLastError();
}

size_t dense_work_size() { return sizeof(DenseWork); }
int dense_tile() { return kDTile; }
int dense_kchunk() { return kDK; }
uint32_t dense_split_rows() { return kDSplitRows; }

void dense_work_fill(void *dst, int8_t *Dt, const uint32_t *count, uint32_t cap, uint32_t stride, int N, int nt, int S,
                     int32_t *P)
{
    DenseWork w{Dt, count, cap, stride, N, nt, S, P};
    *reinterpret_cast<DenseWork *>(dst) = w;
}

}  // namespace gk
