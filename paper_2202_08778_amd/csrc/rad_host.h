// rad_host.h -- host-side helpers shared by the library's translation units:
// error reporting, parameter validation, workspace alignment.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>

#include "../../include/vettam_rad.h"
#include "rad_device.h"

namespace vr {

// Record a thread-local error message and return the status code.
int fail(int status, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();
int check_params(const rad_params_t *p);
// VETTAM_RAD_TRACE=1 in the environment: per-iteration solver trace on stderr
bool trace_enabled();

__host__ __device__ inline size_t align_up(size_t b) { return (b + 255) & ~size_t(255); }

// Kernel-class profiler (see rad_profile_* in the C ABI).  prof_begin returns a
// token (-1 when profiling is off); prof_end records the closing event and the
// launch's algorithmic bytes; prof_resolve turns pending event pairs into times
// (call after the stream has been synchronised).
int prof_begin(int kid, hipStream_t st);
void prof_end(int token, hipStream_t st, double bytes);
void prof_resolve();

// Autotune cache: one "key<TAB>value" line per tuned configuration in
// $VETTAM_RAD_CACHE_DIR/autotune.txt (else ~/.cache/vettam_rad/autotune.txt).
// The last line with a key wins.  device_tag() names the GPU (architecture
// and compute-unit count) for use in keys.
bool cache_get(const std::string &key, std::string &value);
void cache_put(const std::string &key, const std::string &value);
std::string device_tag();

// rad_step on a caller-chosen host staging buffer of kStagingDoubles doubles
// for the reduction read-backs (nullptr: the library's pinned buffer).
constexpr int kStagingDoubles = 256;
int step_with_staging(int nx, int ny, int nz, double *E, double *F, double *T_gas, const void *rho,
                      const void *kappa_P, const void *kappa_R, const void *f_ij, double dt, double dx,
                      const int bc[6], const rad_params_t *p, void *workspace, size_t ws_bytes, void *stream,
                      rad_stats_t *stats, double *host);

enum {
    K_SETUP = 0, K_RESIDUAL, K_APPLY32, K_APPLY64, K_MULTIDOT32, K_MULTIDOT64, K_ORTH32, K_ORTH64,
    K_UPDATEX32, K_UPDATEX64, K_EXCHANGE, K_COMMIT, K_REDUCE, K_BATCHED, K_CLOSURE, K_AMR, K_MG, K_NCLASS
};

}  // namespace vr

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return ::vr::fail(RAD_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define RAD_TRY(expr)               \
    do {                            \
        int r_ = (expr);            \
        if (r_ != RAD_OK) return r_; \
    } while (0)
