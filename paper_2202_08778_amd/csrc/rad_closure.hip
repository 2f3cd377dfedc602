// rad_closure.hip -- local closures that produce the Eddington tensor f_ij
// from the time-lagged radiation state (gfx950).
//
// Sec. 4.1 compares the ray-traced tensor with two local closures evaluated
// from E and F at the start of the step: the Eddington approximation
// f = I/3 and the M1 closure
//   f = (1 - chi)/2 I + (3 chi - 1)/2 n n,  n = F/|F|,
//   chi = (3 + 4 g^2) / (5 + 2 sqrt(4 - 3 g^2)),  g = |F| / (c E).
// One streaming pass, FP64 arithmetic: n n is formed as F_i F_j / |F|^2, so a
// cell needs one square root and one reciprocal.  Where the paper is silent:
// g^2 is clipped to [0, 1]; E <= 0 counts as g = 1 with a flux and g = 0
// without; with F = 0 the n n weight (3 chi - 1)/2 vanishes (chi(0) = 1/3).
#include "rad_host.h"

#include <hip/hip_runtime.h>

#include <cmath>

using namespace vr;

namespace {

template <class OT>
__global__ void __launch_bounds__(256)
    k_closure(long long n, int kind, double c, const double *__restrict__ E, const double *__restrict__ F,
              OT *__restrict__ f)
{
    const long long step = (long long)gridDim.x * 256;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += step) {
        double t[6] = {1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0, 0.0, 0.0, 0.0};
        if (kind == RAD_CLOSURE_M1) {
            const double Fv[3] = {F[i], F[n + i], F[2 * n + i]};
            const double F2 = Fv[0] * Fv[0] + Fv[1] * Fv[1] + Fv[2] * Fv[2];
            const double e = E[i];
            double g2 = e > 0.0 ? F2 / (c * c * e * e) : (F2 > 0.0 ? 1.0 : 0.0);
            g2 = fmin(g2, 1.0);
            const double chi = (3.0 + 4.0 * g2) / (5.0 + 2.0 * sqrt(4.0 - 3.0 * g2));
            const double a = 0.5 * (1.0 - chi);
            const double b = F2 > 0.0 ? 0.5 * (3.0 * chi - 1.0) / F2 : 0.0;
            t[0] = a + b * Fv[0] * Fv[0];
            t[1] = a + b * Fv[1] * Fv[1];
            t[2] = a + b * Fv[2] * Fv[2];
            t[3] = b * Fv[0] * Fv[1];
            t[4] = b * Fv[0] * Fv[2];
            t[5] = b * Fv[1] * Fv[2];
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) f[q * n + i] = (OT)t[q];
    }
}

}  // namespace

extern "C" int rad_closure(long long ncells, const double *E, const double *F, int kind, double c, void *f_ij,
                           int out_dtype, void *stream)
{
    clear_error();
    if (ncells < 0) return fail(RAD_EINVAL, "ncells must be >= 0");
    if (kind != RAD_CLOSURE_EDDINGTON && kind != RAD_CLOSURE_M1) return fail(RAD_EINVAL, "unknown closure kind %d", kind);
    if (!(c > 0) || !std::isfinite(c)) return fail(RAD_EINVAL, "c must be positive and finite");
    if (out_dtype != RAD_F64 && out_dtype != RAD_F32) return fail(RAD_EINVAL, "unknown output dtype %d", out_dtype);
    if (ncells == 0) return RAD_OK;
    if (!E || !F || !f_ij) return fail(RAD_EINVAL, "NULL data pointer");
    hipStream_t st = (hipStream_t)stream;
    const long long blocks = std::min<long long>((ncells + 255) / 256, 65536);
    const int tok = prof_begin(K_CLOSURE, st);
    if (out_dtype == RAD_F64)
        hipLaunchKernelGGL(k_closure<double>, dim3((unsigned)blocks), dim3(256), 0, st, ncells, kind, c, E, F,
                           (double *)f_ij);
    else
        hipLaunchKernelGGL(k_closure<float>, dim3((unsigned)blocks), dim3(256), 0, st, ncells, kind, c, E, F,
                           (float *)f_ij);
    HIP_TRY(hipGetLastError());
    // reads E (and F for M1), writes six tensor planes
    prof_end(tok, st, (double)ncells * ((kind == RAD_CLOSURE_M1 ? 32 : 0) + 6.0 * (out_dtype == RAD_F64 ? 8 : 4)));
    return RAD_OK;
}
