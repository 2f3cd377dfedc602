// rad_noalloc.hip -- rad_step_noalloc: rad_step for callers that cannot
// allocate (code under HIP graph capture, serving loops, harnesses that forbid
// hipMalloc).  Its workspace is the file-scope device array `scratch` below:
// one copy per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in symbol): the
// device address of the current device's copy is looked up once per device
// with hipGetSymbolAddress and that pointer is handed to the step as its
// workspace.  The reductions' results come back through a thread-local
// pageable host buffer, so the call makes no device or pinned allocation.
// Every call on one GPU shares that GPU's array; calls that overlap on one
// GPU (other host threads, other streams) race.  The step writes every
// workspace value before reading it, so the array needs no clearing between
// calls.
#include "rad_host.h"

#include <cstring>
#include <mutex>

using namespace vr;

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;   // 64 MiB per GPU
constexpr int kMaxDevices = 64;

__device__ __attribute__((aligned(256))) char scratch[kScratchBytes];

std::mutex g_mu;
void *g_addr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (looked up on the
// first call on that device, with the device current).
int scratch_address(void **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(RAD_EINVAL, "device index %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[dev]) {
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(RAD_EHIP, "no device address for the scratch array");
        g_addr[dev] = ptr;
    }
    *out = g_addr[dev];
    return RAD_OK;
}

}  // namespace

extern "C" size_t rad_noalloc_max_bytes(void) { return kScratchBytes; }

extern "C" int rad_step_noalloc(int nx, int ny, int nz, double *E, double *F, double *T_gas, const void *rho,
                                const void *kappa_P, const void *kappa_R, const void *f_ij, double dt, double dx,
                                const int bc[6], const rad_params_t *p, void *stream, rad_stats_t *stats)
{
    clear_error();
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (!p) return fail(RAD_EINVAL, "params is NULL");
    const size_t need = rad_workspace_bytes(nx, ny, nz, p);
    if (need == 0) {   // invalid arguments: let the step name the reason
        return step_with_staging(nx, ny, nz, E, F, T_gas, rho, kappa_P, kappa_R, f_ij, dt, dx, bc, p, nullptr, 0,
                                 stream, stats, nullptr);
    }
    if (need > kScratchBytes)
        return fail(RAD_ENOMEM, "rad_step_noalloc: the step needs %zu bytes of workspace, the scratch holds %zu",
                    need, kScratchBytes);
    void *ws = nullptr;
    RAD_TRY(scratch_address(&ws));
    static thread_local double host[kStagingDoubles];
    return step_with_staging(nx, ny, nz, E, F, T_gas, rho, kappa_P, kappa_R, f_ij, dt, dx, bc, p, ws, kScratchBytes,
                             stream, stats, host);
}
