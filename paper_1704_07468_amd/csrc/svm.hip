// Training consumer of the kernel: the support-vector machine of Eq. 1
// (Section 3.1 trains an SVM on the gapped k-mer Gram matrix) by dual
// coordinate descent on the normalised kernel.
//
// The bias is absorbed into the kernel (K' = K + 1, so b = sum_i alpha_i y_i)
// and the box-constrained dual
//     minimise 1/2 alpha^T Q alpha - sum_i alpha_i,  0 <= alpha_i <= C,
//     Q_ij = y_i y_j K'_ij
// is solved one coordinate at a time (Hsieh et al., ICML 2008): coordinate i
// moves to the clipped minimiser along it, alpha_i <- clip(alpha_i - G_i /
// Q_ii, 0, C) with G = Q alpha - 1, and G is updated by d * Q[:, i].  The
// coordinates are visited in the order 0..N-1; a run stops after the first
// epoch whose projected gradients span at most eps, or after max_epochs.
//
// The method is sequential over coordinates, so one block runs it: each
// thread owns PER columns j (j = tid + p * NT) and keeps their G_j, alpha_j
// and y_j in registers; at step i the owner of column i publishes (G_i,
// alpha_i, K_ii, y_i) in one of two LDS slots (one barrier per step), every
// thread computes the same update from it, and adds d * Q_ij to its own G_j
// from row i of K, which was loaded during the previous step.  Every FP64
// operation is a separately rounded add, multiply or divide (no contraction),
// in the same order as the plain statement of the method, so that the
// multipliers do not depend on how the work is spread over threads (they
// agree with a sequential host run to about 1e-11 relative).
#include <hip/hip_runtime.h>

#include <cmath>

#include "plan.h"

namespace gk {
void clear_error();
}
using namespace gk;

namespace {

constexpr int kSvmMaxN = 8192;

struct SvmBc {
    double g, a, kii;
    int32_t y, pad;
};

struct SvmInfo {
    double bias;
    int32_t epochs;
    int32_t bad_label;
};

template <int NT, int PER>
__global__ __launch_bounds__(NT) void k_svm_dcd(const double *__restrict__ K, const int8_t *__restrict__ y, int N, double C,
                                                double eps, int max_epochs, double *alpha_out, double *dual_out,
                                                SvmInfo *info)
{
    __shared__ SvmBc bc[2];
    __shared__ int bad;
    extern __shared__ double dual_lds[];
    const int tid = threadIdx.x;
    double G[PER], A[PER], R[PER];
    int Y[PER];
    if (tid == 0) bad = 0;
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int j = tid + p * NT;
        G[p] = 0.0;
        A[p] = 0.0;
        Y[p] = 1;
        R[p] = 0.0;
        if (j < N) {
            Y[p] = y[j];
            if (Y[p] != 1 && Y[p] != -1) atomicOr(&bad, 1);
            R[p] = K[j];  // row 0
        }
    }
    __syncthreads();
    if (bad) {
        if (tid == 0) info->bad_label = 1;
        return;  // block-uniform
    }
    if (tid == 0) bc[0] = SvmBc{G[0], A[0], R[0], Y[0], 0};
    uint32_t step = 0;
    int ep = 0;
    while (ep < max_epochs) {
        double pgmax = -HUGE_VAL, pgmin = HUGE_VAL;
        for (int i = 0; i < N; ++i, ++step) {
            __syncthreads();  // bc[step & 1] holds coordinate i
            const SvmBc b = bc[step & 1];
            // the next row is loaded now and used in the next step
            const int inext = i + 1 < N ? i + 1 : 0;
            double Rn[PER];
#pragma unroll
            for (int p = 0; p < PER; ++p) {
                const int j = tid + p * NT;
                Rn[p] = j < N ? K[(size_t)inext * N + j] : 0.0;
            }
            const double qii = __dadd_rn(b.kii, 1.0);
            const double g = __dadd_rn(b.g, -1.0);
            double pg = g;
            if (b.a == 0.0) pg = fmin(g, 0.0);
            else if (b.a == C) pg = fmax(g, 0.0);
            pgmax = fmax(pgmax, pg);
            pgmin = fmin(pgmin, pg);
            if (pg != 0.0) {
                const double a_new = fmin(fmax(__dadd_rn(b.a, -__ddiv_rn(g, qii)), 0.0), C);
                const double d = __dadd_rn(a_new, -b.a);
                if (tid == i % NT) {
#pragma unroll
                    for (int p = 0; p < PER; ++p)
                        if (p == i / NT) A[p] = a_new;
                }
                if (d != 0.0) {
#pragma unroll
                    for (int p = 0; p < PER; ++p) {
                        double q = __dadd_rn(R[p], 1.0);
                        if (Y[p] != b.y) q = -q;
                        G[p] = __dadd_rn(G[p], __dmul_rn(d, q));
                    }
                }
            }
#pragma unroll
            for (int p = 0; p < PER; ++p) R[p] = Rn[p];
            if (tid == inext % NT) {
#pragma unroll
                for (int p = 0; p < PER; ++p)
                    if (p == inext / NT) bc[(step + 1) & 1] = SvmBc{G[p], A[p], R[p], Y[p], 0};
            }
        }
        ++ep;
        if (pgmax - pgmin <= eps) break;  // the same values in every thread
    }
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int j = tid + p * NT;
        if (j < N) {
            const double dv = A[p] * (double)Y[p];
            if (alpha_out) alpha_out[j] = A[p];
            if (dual_out) dual_out[j] = dv;
            dual_lds[j] = dv;
        }
    }
    __syncthreads();
    if (tid == 0) {
        double bsum = 0.0;  // ascending order
        for (int j = 0; j < N; ++j) bsum = __dadd_rn(bsum, dual_lds[j]);
        info->bias = bsum;
        info->epochs = ep;
        info->bad_label = 0;
    }
}

template <int NT, int PER>
hipError_t launch_svm(const double *K, const int8_t *y, int N, double C, double eps, int max_epochs, double *alpha,
                      double *dual, SvmInfo *info, hipStream_t st)
{
    hipLaunchKernelGGL((k_svm_dcd<NT, PER>), dim3(1), dim3(NT), (size_t)N * sizeof(double), st, K, y, N, C, eps,
                       max_epochs, alpha, dual, info);
    return hipGetLastError();
}

}  // namespace

extern "C" {

gakco_status gakco_svm_train(gakco_ctx *ctx, const double *K, const int8_t *y, int32_t N, double C, double eps,
                             int32_t max_epochs, double *alpha_out, double *dual_coef_out, double *bias_out,
                             int32_t *epochs_out, void *hip_stream)
{
    clear_error();
    if (!ctx || !K || !y) { set_error("ctx, K and y must not be NULL"); return GAKCO_EINVAL; }
    if (N < 1 || !(C > 0.0) || !(eps >= 0.0) || max_epochs < 1) {
        set_error("need N >= 1, C > 0, eps >= 0, max_epochs >= 1 (got N=%d, C=%g, eps=%g, max_epochs=%d)", N, C, eps,
                  max_epochs);
        return GAKCO_EINVAL;
    }
    if (N > kSvmMaxN) {
        set_error("N=%d exceeds the single-block solver's %d coordinates", N, kSvmMaxN);
        return GAKCO_EUNSUPPORTED;
    }
    GK_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    void *small = nullptr;
    GK_TRY(ctx_small_buffer(ctx, &small));
    SvmInfo *info = static_cast<SvmInfo *>(small);
    GK_HIP(launch_fill_u32(reinterpret_cast<uint32_t *>(info), sizeof(SvmInfo) / 4, 0u, st));
    if (N <= 256) GK_HIP((launch_svm<256, 1>(K, y, N, C, eps, max_epochs, alpha_out, dual_coef_out, info, st)));
    else if (N <= 1024) GK_HIP((launch_svm<256, 4>(K, y, N, C, eps, max_epochs, alpha_out, dual_coef_out, info, st)));
    else if (N <= 2048) GK_HIP((launch_svm<256, 8>(K, y, N, C, eps, max_epochs, alpha_out, dual_coef_out, info, st)));
    else GK_HIP((launch_svm<1024, 8>(K, y, N, C, eps, max_epochs, alpha_out, dual_coef_out, info, st)));
    SvmInfo h{};
    GK_HIP(hipMemcpyAsync(&h, info, sizeof h, hipMemcpyDeviceToHost, st));
    GK_HIP(hipStreamSynchronize(st));
    if (h.bad_label) { set_error("a label is neither +1 nor -1"); return GAKCO_EINVAL; }
    if (bias_out) *bias_out = h.bias;
    if (epochs_out) *epochs_out = h.epochs;
    return GAKCO_OK;
}

}  // extern "C"
