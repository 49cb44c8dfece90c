// Allocation-free variant of goac_energies for callers that cannot allocate
// device memory (code under stream capture, tight serving loops, harnesses that
// forbid allocation). Its scratch is a fixed file-scope device array, which every
// GPU the library runs on holds for the life of the process.
//
// Host code never passes the array's name to a kernel: in host code the name is a
// host-side stand-in, not a device address. The device address comes from
// hipGetSymbolAddress, looked up once per device with that device current (at
// context creation) and kept per device.
#include <mutex>

#include "common.h"

namespace goac {

// scratch of goac_energies_noalloc: the check word, then the energies' buffers
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
constexpr size_t kNoAllocFlagBytes = 256;
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kNoAllocMaxDevices] = {};

hipError_t noalloc_setup(int device) {
    if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = ptr;
    return hipSuccess;
}

// clears the check word
__global__ void k_clear_flag(int32_t* flag) {
    if (threadIdx.x == 0) *flag = 0;
}

static void* scratch_of(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return (device >= 0 && device < kNoAllocMaxDevices) ? g_scratch_ptr[device] : nullptr;
}

}  // namespace goac

using namespace goac;

extern "C" goac_status goac_energies_noalloc(goac_problem* pb, int64_t P, const uint8_t* occ, goac_precision prec,
                                             double* E) {
    if (!pb) return GOAC_EINVAL;
    goac_ctx* ctx = pb->ctx;
    if (P < 0 || P > ((int64_t)1 << 30) || (P > 0 && (!occ || !E)))
        return fail(ctx, GOAC_EINVAL, "energies_noalloc: bad arguments");
    if (prec != GOAC_FP64 && prec != GOAC_MIXED) return fail(ctx, GOAC_EINVAL, "energies_noalloc: unknown precision");
    if (prec == GOAC_MIXED && !pb->d.mixed_exact)
        return fail(ctx, GOAC_EINEXACT, "energies_noalloc: a shifted charge is not bf16-exact");
    if (P == 0) return GOAC_OK;
    const size_t need = energies_scratch_bytes(pb, P, prec);
    if (need > kNoAllocScratchBytes - kNoAllocFlagBytes)
        return fail(ctx, GOAC_EINVAL,
                    "energies_noalloc: " + std::to_string(P) + " rows need " + std::to_string(need) +
                        " bytes of scratch, more than the fixed " +
                        std::to_string(kNoAllocScratchBytes - kNoAllocFlagBytes));
    GOAC_HIP(ctx, hipSetDevice(ctx->device));
    char* base = (char*)scratch_of(ctx->device);
    if (!base) return fail(ctx, GOAC_EHIP, "energies_noalloc: no scratch address for this device");
    int32_t* flag = (int32_t*)base;
    // the check (it clears the flag first), then the energy kernels, which skip all
    // work when the check failed
    WsSource src{ctx, base + kNoAllocFlagBytes, kNoAllocScratchBytes - kNoAllocFlagBytes, 0};
    if (prec == GOAC_MIXED) {
        // the mixed path's row kernel checks the rows as it reads them
        hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, ctx->stream, flag);
        GOAC_CHECK_LAUNCH(ctx);
        GOAC_TRY(energies_mixed(pb, P, occ, E, 0, flag, &src));
    } else {
        GOAC_TRY(rows_check_launch(pb, P, occ, flag));
        GOAC_TRY(energies_fp64(pb, P, occ, E, flag, &src));
    }
    int32_t bad = 0;
    GOAC_HIP(ctx, hipMemcpyAsync(&bad, flag, sizeof bad, hipMemcpyDeviceToHost, ctx->stream));
    GOAC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (bad)
        return fail(ctx, GOAC_EINVAL,
                    "energies_noalloc: an occupation holds an unknown species or breaks the problem's composition");
    return GOAC_OK;
}
