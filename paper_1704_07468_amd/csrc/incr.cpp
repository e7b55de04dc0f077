// Incremental Gram: a kernel matrix that grows as sequences are appended,
// each append computing only the new rows (Section 3.2 notes that the
// counting approach suits adaptive training, where the set grows).
//
// The sequences appended so far are kept as resident segments, one per
// append (their per-position-set group tables, as for serving).  Appending n
// sequences to N:
//   * their rows against every earlier segment come from the serving join
//     (kernel rows of the new sequences as queries), written straight into
//     the lower-left block of the new (N+n) x (N+n) matrix;
//   * their own n x n block is a Gram of the new sequences;
//   * the old N x N block is copied from the previous matrix and the
//     upper-right block mirrored from the lower-left one;
//   * the new sequences become one more segment.
// Every entry is the one the Gram of all N+n sequences gives: C_m, N_m and K
// are exact integers per pair, and the normalisation divides by the same
// sqrt(K_xx K_yy) (older sequence first) as the Gram's epilogue.
#include <vector>

#include "plan.h"

namespace gk {
void clear_error();
hipError_t init_rows_attributes(size_t lds);
}  // namespace gk
using namespace gk;

struct gakco_incr {
    gakco_ctx *ctx = nullptr;
    int32_t sigma = 0, g = 0, k = 0;
    int64_t N = 0;
    std::vector<gakco_resident *> segs;
    std::vector<int64_t> seg_off;
    double *kblk = nullptr;  // the new sequences' own block (grow-only)
    size_t kblk_cap = 0;
};

extern "C" {

gakco_status gakco_incr_create(gakco_ctx *ctx, int32_t sigma, int32_t g, int32_t k, gakco_incr **out)
{
    clear_error();
    if (!ctx || !out) { set_error("ctx/out is NULL"); return GAKCO_EINVAL; }
    *out = nullptr;
    if (sigma < 1 || sigma > 127 || g < 1 || k < 0 || k > g) {
        set_error("need 1 <= sigma <= 127, g >= 1, 0 <= k <= g (got sigma=%d, g=%d, k=%d)", sigma, g, k);
        return GAKCO_EINVAL;
    }
    if (g * symbol_bits(sigma) > 64) { set_error("g*b exceeds the 64-bit packed g-mer"); return GAKCO_EUNSUPPORTED; }
    auto *inc = new gakco_incr();
    inc->ctx = ctx;
    inc->sigma = sigma;
    inc->g = g;
    inc->k = k;
    *out = inc;
    return GAKCO_OK;
}

void gakco_incr_destroy(gakco_incr *inc)
{
    if (!inc) return;
    for (auto *r : inc->segs) gakco_resident_destroy(r);
    if (inc->kblk) {
        (void)hipSetDevice(inc->ctx->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(inc->kblk);
    }
    delete inc;
}

gakco_status gakco_incr_info(const gakco_incr *inc, int64_t *N, int32_t *segments)
{
    clear_error();
    if (!inc) { set_error("incr is NULL"); return GAKCO_EINVAL; }
    if (N) *N = inc->N;
    if (segments) *segments = (int32_t)inc->segs.size();
    return GAKCO_OK;
}

gakco_status gakco_incr_append(gakco_incr *inc, const int8_t *seqs, const int32_t *lens, int32_t n_new,
                               const double *K_prev, double *K_out, void *hip_stream)
{
    clear_error();
    if (!inc || !seqs || !lens || !K_out || n_new < 1) {
        set_error("need incr, seqs, lens, K_out and n_new >= 1");
        return GAKCO_EINVAL;
    }
    const int64_t N0 = inc->N, Nt = N0 + n_new;
    if (N0 > 0 && !K_prev) { set_error("K_prev is NULL but %lld sequences are there", (long long)N0); return GAKCO_EINVAL; }
    if (N0 > 0 && K_prev == K_out) { set_error("K_prev and K_out must not be the same buffer"); return GAKCO_EINVAL; }
    if (Nt > (1 << 24)) { set_error("more than 2^24 sequences"); return GAKCO_EUNSUPPORTED; }
    gakco_ctx *ctx = inc->ctx;
    GK_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    // the new block, a Gram of the new sequences (validates them)
    const size_t blk = (size_t)n_new * (size_t)n_new * sizeof(double);
    if (blk > inc->kblk_cap) {
        if (inc->kblk) {
            GK_HIP(hipStreamSynchronize(st));
            GK_HIP(hipFree(inc->kblk));
            inc->kblk = nullptr;
            inc->kblk_cap = 0;
        }
        GK_HIP(hipMalloc(&inc->kblk, blk));
        inc->kblk_cap = blk;
    }
    GK_TRY(gakco_gram(ctx, seqs, lens, n_new, inc->sigma, inc->g, inc->k, inc->kblk, nullptr, nullptr, hip_stream));
    // their rows against every earlier segment, into the lower-left block
    if (!inc->segs.empty()) GK_HIP(init_rows_attributes(ctx->lds_max));
    for (size_t s = 0; s < inc->segs.size(); ++s)
        GK_TRY(rows_run(ctx, inc->segs[s], seqs, lens, nullptr, n_new, K_out + (size_t)N0 * Nt + inc->seg_off[s], Nt,
                        nullptr, nullptr, st));
    // old block, new block, upper-right mirror
    if (N0 > 0)
        GK_HIP(hipMemcpy2DAsync(K_out, (size_t)Nt * 8, K_prev, (size_t)N0 * 8, (size_t)N0 * 8, (size_t)N0,
                                hipMemcpyDeviceToDevice, st));
    GK_HIP(hipMemcpy2DAsync(K_out + (size_t)N0 * Nt + N0, (size_t)Nt * 8, inc->kblk, (size_t)n_new * 8,
                            (size_t)n_new * 8, (size_t)n_new, hipMemcpyDeviceToDevice, st));
    GK_HIP(launch_mirror_block(K_out, Nt, (int)N0, (int)N0, n_new, st));
    // the new sequences become a segment for later appends
    gakco_resident *seg = nullptr;
    GK_TRY(gakco_resident_create(ctx, seqs, lens, n_new, inc->sigma, inc->g, inc->k, nullptr, 0.0, &seg));
    inc->segs.push_back(seg);
    inc->seg_off.push_back(N0);
    inc->N = Nt;
    GK_HIP(hipStreamSynchronize(st));
    return GAKCO_OK;
}

}  // extern "C"
