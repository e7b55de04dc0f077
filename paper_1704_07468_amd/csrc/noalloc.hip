// Gram entry point for callers that cannot allocate device memory.
//
// Its scratch (g-mer arrays, partition and sort pool, count matrices, split
// partial tiles, descriptor blob, flags) lives in one file-scope device array
// that every GPU the library runs on holds from load until the process ends.
// Host code never passes that array's name to a kernel or a copy: the name is
// a host-side stand-in; the array's device address on each GPU comes from
// hipGetSymbolAddress, taken once per device with that device current, and
// only that address is handed to the planner.
#include <mutex>

#include "plan.h"

namespace gk {
hipError_t init_kernel_attributes(size_t acc_lds);
void clear_error();
}  // namespace gk

using namespace gk;

namespace {

constexpr size_t kNoAllocScratchBytes = 512ull << 20;  // GAKCO_NOALLOC_SCRATCH_BYTES
static_assert(kNoAllocScratchBytes == (size_t)GAKCO_NOALLOC_SCRATCH_BYTES, "header and library disagree");

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;

// Per device: the array's address and a context bound to it (no side stream,
// no profiler, nothing that allocates).  The mutex serialises this library's
// calls on the device, which share the array.
struct DeviceScratch {
    std::mutex mu;
    bool ready = false;
    void *ptr = nullptr;
    gakco_ctx ctx;
};
DeviceScratch g_dev[kMaxDevices];

gakco_status setup(DeviceScratch &d, int device)
{
    if (d.ready) return GAKCO_OK;
    void *ptr = nullptr;
    GK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) { set_error("hipGetSymbolAddress returned no address for the scratch array"); return GAKCO_EHIP; }
    int lds = 0;
    GK_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    gakco_ctx &c = d.ctx;
    c.device = device;
    c.budget = kNoAllocScratchBytes;
    c.dense_tau = 192;
    c.lds_max = (size_t)lds > 8192 ? (size_t)lds - 8192 : 0;
    c.overlap = false;
    c.side = nullptr;
    c.fixed_arena = true;
    c.arena = ptr;
    c.arena_cap = kNoAllocScratchBytes;
    c.pool_cap = kNoAllocScratchBytes;
    if (init_kernel_attributes(c.lds_max) != hipSuccess) { set_error("hipFuncSetAttribute failed"); return GAKCO_EHIP; }
    d.ptr = ptr;
    d.ready = true;
    return GAKCO_OK;
}

}  // namespace

extern "C" gakco_status gakco_gram_noalloc(const int8_t *seqs, const int32_t *lens, int32_t N, int32_t sigma, int32_t g,
                                           int32_t k, double *K_out, int64_t *Nm_out, int64_t *Cm_out,
                                           void *hip_stream)
{
    clear_error();
    int device = -1;
    GK_HIP(hipGetDevice(&device));
    if (device < 0 || device >= kMaxDevices) { set_error("device %d beyond the %d supported", device, kMaxDevices); return GAKCO_EUNSUPPORTED; }
    if (N < 1) { set_error("N must be >= 1 (got %d)", N); return GAKCO_EINVAL; }
    if (!seqs || !lens) { set_error("seqs and lens must not be NULL"); return GAKCO_EINVAL; }
    DeviceScratch &d = g_dev[device];
    std::lock_guard<std::mutex> lock(d.mu);
    GK_TRY(setup(d, device));
    gakco_ctx *ctx = &d.ctx;
    hipStream_t st = (hipStream_t)hip_stream;
    Plan p;
    p.jobs.resize(1);
    JobPlan &jp = p.jobs[0];
    jp.seqs = seqs; jp.lens_dev = lens; jp.N = N; jp.sigma = sigma; jp.g = g; jp.k = k;
    jp.K_out = K_out; jp.Nm_out = Nm_out; jp.Cm_out = Cm_out;
    GK_TRY(fetch_lens(jp, st));
    GK_TRY(plan_shape(ctx, jp, nullptr, 0));
    return run_single(ctx, p, st);
}
