// int8 matrix-core path of the count update (Algorithm 1 countAndUpdate) for
// groups with many distinct sequences.
//
// Each such group of a level m is one row r of a count matrix D_m (row r,
// column X = how often sequence X holds the group's reduced g-mer), so the
// group's contribution to C_m is the outer product of that row with itself
// and the contribution of all of them is D_m^T D_m.  Counts are <= 127, so
// int8 operands with int32 accumulation are exact for up to
// 2^31 / 127^2 = 133144 rows; partial sums are added into the int64 C_m every
// 65536 rows.  D is stored sequence-major (Dt[X][r]) so every MFMA operand
// is 16 contiguous bytes along r.  Only tiles on or above the diagonal are
// computed; the epilogue mirrors the upper triangle.
#include "common.h"
#include "launch.h"

namespace gk {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kDTile = 128;           // output tile edge
constexpr uint32_t kDFlush = 65536;   // rows per exact int32 partial sum

struct DenseWork {
    int8_t *Dt;              // [Npad][stride] counts, zero beyond the used rows
    const uint32_t *count;   // rows used (device counter)
    uint32_t cap;            // row capacity
    uint32_t stride;         // bytes per sequence (multiple of 32, >= cap)
    int32_t N, nt;           // sequences, tiles per edge
    int64_t *C;              // C_m [N][N]
};

// v_mfma_i32_32x32x32_i8 operand layout: lane l supplies row/column (l % 32)
// and 16 consecutive k values starting at 16*(l/32); accumulator v of lane l
// is element (8*(v/4) + 4*(l/32) + v%4, l % 32).
__global__ __launch_bounds__(kThreads) void k_dense_syrk(const DenseWork *__restrict__ dw, const uint32_t *__restrict__ bprefix,
                                                         int nwork)
{
    const int wi = find_item(bprefix, nwork, blockIdx.x);
    const DenseWork &W = dw[wi];
    const uint32_t R = min(*W.count, W.cap);
    if (R == 0) return;
    // flat upper-tile index -> (I, J), I <= J
    int f = (int)(blockIdx.x - bprefix[wi]);
    int I = 0;
    while (f >= W.nt - I) {
        f -= W.nt - I;
        ++I;
    }
    const int J = I + f;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wx = wave & 1, wy = wave >> 1;
    const int x0 = I * kDTile + wx * 64, y0 = J * kDTile + wy * 64;
    const int8_t *pa0 = W.Dt + (size_t)(x0 + (lane & 31)) * W.stride + 16 * (lane >> 5);
    const int8_t *pa1 = pa0 + (size_t)32 * W.stride;
    const int8_t *pb0 = W.Dt + (size_t)(y0 + (lane & 31)) * W.stride + 16 * (lane >> 5);
    const int8_t *pb1 = pb0 + (size_t)32 * W.stride;
    const int N = W.N;
    for (uint32_t r0 = 0; r0 < R; r0 += kDFlush) {
        const uint32_t r1 = min(R, r0 + kDFlush);
        v16i acc00 = {}, acc01 = {}, acc10 = {}, acc11 = {};
        for (uint32_t r = r0; r < r1; r += 32) {
            const v4i a0 = *reinterpret_cast<const v4i *>(pa0 + r);
            const v4i a1 = *reinterpret_cast<const v4i *>(pa1 + r);
            const v4i b0 = *reinterpret_cast<const v4i *>(pb0 + r);
            const v4i b1 = *reinterpret_cast<const v4i *>(pb1 + r);
            acc00 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, b0, acc00, 0, 0, 0);
            acc01 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, b1, acc01, 0, 0, 0);
            acc10 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, b0, acc10, 0, 0, 0);
            acc11 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, b1, acc11, 0, 0, 0);
        }
        auto flush = [&](const v16i &acc, int xb, int yb) {
            const int y = yb + (lane & 31);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int x = xb + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                if (x < N && y < N && x <= y && acc[v]) W.C[(size_t)x * N + y] += (int64_t)acc[v];
            }
        };
        flush(acc00, x0, y0);
        flush(acc01, x0, y0 + 32);
        flush(acc10, x0 + 32, y0);
        flush(acc11, x0 + 32, y0 + 32);
    }
}

// Restore the zero invariant of Dt: clear the used rows of every sequence.
__global__ __launch_bounds__(kThreads) void k_dense_clear(const DenseWork *__restrict__ dw, int nwork)
{
    const DenseWork &W = dw[blockIdx.y];
    const uint32_t R = min(*W.count, W.cap);
    const uint32_t nv = (R + 15) / 16;  // 16-byte words per sequence row (stride is a multiple of 32)
    const size_t total = (size_t)W.N * nv;
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < total; i += (size_t)gridDim.x * kThreads) {
        const size_t x = i / nv, q = i - x * nv;
        *reinterpret_cast<v4i *>(W.Dt + x * W.stride + q * 16) = v4i{0, 0, 0, 0};
    }
    (void)nwork;
}

hipError_t launch_dense(const DenseWork *dw, const uint32_t *bprefix, int nwork, uint32_t nblocks, hipStream_t st)
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

void dense_work_fill(void *dst, int8_t *Dt, const uint32_t *count, uint32_t cap, uint32_t stride, int N, int nt,
                     int64_t *C)
{
    DenseWork w{Dt, count, cap, stride, N, nt, C};
    *reinterpret_cast<DenseWork *>(dst) = w;
}

}  // namespace gk
