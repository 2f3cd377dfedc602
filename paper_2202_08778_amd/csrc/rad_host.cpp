// rad_host.cpp -- error state, defaults, parameter checks, profiler and autotune cache of the C ABI.
#include "rad_host.h"

#ifndef VETTAM_BUILD_ID
#define VETTAM_BUILD_ID "unknown"
#endif

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <string>
#include <vector>

#include <sys/stat.h>

namespace vr {

static thread_local std::string g_err;

int fail(int status, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return status;
}

void clear_error() { g_err.clear(); }

bool trace_enabled()
{
    static const bool on = [] {
        const char *v = std::getenv("VETTAM_RAD_TRACE");
        return v && v[0] && v[0] != '0';
    }();
    return on;
}

int check_params(const rad_params_t *p)
{
    if (!p) return fail(RAD_EINVAL, "params is NULL");
    if (!(p->c > 0) || !std::isfinite(p->c)) return fail(RAD_EINVAL, "c must be positive and finite");
    if (!(p->a_R >= 0) || !std::isfinite(p->a_R)) return fail(RAD_EINVAL, "a_R must be >= 0 and finite");
    if (!(p->c_v >= 0) || !std::isfinite(p->c_v)) return fail(RAD_EINVAL, "c_v must be >= 0 and finite");
    if (!(p->tol > 0)) return fail(RAD_EINVAL, "tol must be positive");
    if (!(p->eps_R > 0)) return fail(RAD_EINVAL, "eps_R must be positive");
    if (!(p->eps_P >= 0)) return fail(RAD_EINVAL, "eps_P must be >= 0");
    if (p->max_picard < 1) return fail(RAD_EINVAL, "max_picard must be >= 1");
    if (p->max_krylov < 1) return fail(RAD_EINVAL, "max_krylov must be >= 1");
    if (p->gmres_m < 1 || p->gmres_m > kMaxM) return fail(RAD_EINVAL, "gmres_m must be in [1, %d]", kMaxM);
    if (p->prec != RAD_FP64 && p->prec != RAD_MIXED) return fail(RAD_EINVAL, "unknown precision %d", p->prec);
    if (p->mode != RAD_PICARD_LAGGED && p->mode != RAD_PICARD_LINEARISED)
        return fail(RAD_EINVAL, "unknown Picard mode %d", p->mode);
    if (p->coef_dtype != RAD_F64 && p->coef_dtype != RAD_F32)
        return fail(RAD_EINVAL, "unknown coefficient dtype %d", p->coef_dtype);
    if (p->anderson_m < 0 || p->anderson_m > kMaxAnderson)
        return fail(RAD_EINVAL, "anderson_m must be in [0, %d]", kMaxAnderson);
    if (p->vel_implicit != 0 && p->vel_implicit != 1) return fail(RAD_EINVAL, "vel_implicit must be 0 or 1");
    if (p->cv_cubic != 0 && p->cv_cubic != 1) return fail(RAD_EINVAL, "cv_cubic must be 0 or 1");
    if (p->krylov_poly < 0 || p->krylov_poly > 2) return fail(RAD_EINVAL, "krylov_poly must be 0, 1 or 2");
    for (int f = 0; f < 6; ++f)
        if (!std::isfinite(p->F_inc[f])) return fail(RAD_EINVAL, "F_inc[%d] must be finite", f);
    if (!(p->eps_N >= 0) || !(p->eps_N < 1)) return fail(RAD_EINVAL, "eps_N must be in [0, 1)");
    if (p->energy_fix != 0 && p->energy_fix != 1) return fail(RAD_EINVAL, "energy_fix must be 0 or 1");
    if (p->energy_fix && p->anderson_m > 0) return fail(RAD_EINVAL, "energy_fix needs anderson_m = 0");
    if (p->max_refine < 0) return fail(RAD_EINVAL, "max_refine must be >= 0");
    return RAD_OK;
}

// ------------------------------------------------------------------ profiler

static const char *const kNames[K_NCLASS] = {
    "setup", "residual_fp64", "apply_fp32", "apply_fp64", "multidot_fp32", "multidot_fp64", "orth_update_fp32",
    "orth_update_fp64", "update_x_fp32", "update_x_fp64", "exchange_fp64", "commit", "reduce", "batched_persistent",
    "closure", "amr_jump", "multigrid_levels"};

struct Pending {
    hipEvent_t a, b;
    int kid;
    double bytes;
};

static bool g_prof_on = false;
static bool g_prof_apply_only = false;   // events around the operator applies only
static std::vector<Pending> g_pending;
static std::vector<hipEvent_t> g_pool;
static double g_ms[K_NCLASS], g_bytes[K_NCLASS];
static long long g_launch[K_NCLASS];

static hipEvent_t get_event()
{
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int prof_begin(int kid, hipStream_t st)
{
    if (!g_prof_on) return -1;
    Pending p;
    if (g_prof_apply_only && kid != K_APPLY32 && kid != K_APPLY64) {
        // counted (bytes, launches) but not timed: no event on the stream
        p.a = p.b = nullptr;
        p.kid = kid;
        p.bytes = 0;
        g_pending.push_back(p);
        return (int)g_pending.size() - 1;
    }
    p.a = get_event();
    p.b = get_event();
    if (!p.a || !p.b) return -1;
    p.kid = kid;
    p.bytes = 0;
    if (hipEventRecord(p.a, st) != hipSuccess) {
        g_pool.push_back(p.a);
        g_pool.push_back(p.b);
        return -1;
    }
    g_pending.push_back(p);
    return (int)g_pending.size() - 1;
}

void prof_end(int token, hipStream_t st, double bytes)
{
    if (token < 0 || token >= (int)g_pending.size()) return;
    g_pending[token].bytes = bytes;
    if (!g_pending[token].b) return;
    if (hipEventRecord(g_pending[token].b, st) != hipSuccess) g_pending[token].kid = -1;
}

void prof_resolve()
{
    for (auto &p : g_pending) {
        if (!p.a) {
            g_bytes[p.kid] += p.bytes;
            g_launch[p.kid] += 1;
            continue;
        }
        float ms = 0;
        if (p.kid >= 0 && hipEventSynchronize(p.b) == hipSuccess &&
            hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            g_ms[p.kid] += ms;
            g_bytes[p.kid] += p.bytes;
            g_launch[p.kid] += 1;
        }
        g_pool.push_back(p.a);
        g_pool.push_back(p.b);
    }
    g_pending.clear();
}

}  // namespace vr

extern "C" void rad_profile_enable(int on)
{
    vr::g_prof_on = on != 0;
    vr::g_prof_apply_only = on == 2;
}

extern "C" void rad_profile_reset(void)
{
    vr::prof_resolve();
    for (int k = 0; k < vr::K_NCLASS; ++k) {
        vr::g_ms[k] = 0;
        vr::g_bytes[k] = 0;
        vr::g_launch[k] = 0;
    }
}

extern "C" int rad_profile_count(void)
{
    vr::prof_resolve();
    int n = 0;
    for (int k = 0; k < vr::K_NCLASS; ++k) n += vr::g_launch[k] > 0;
    return n;
}

extern "C" int rad_profile_get(int idx, const char **name, double *ms, double *bytes, long long *launches)
{
    vr::prof_resolve();
    int n = 0;
    for (int k = 0; k < vr::K_NCLASS; ++k) {
        if (vr::g_launch[k] == 0) continue;
        if (n++ == idx) {
            if (name) *name = vr::kNames[k];
            if (ms) *ms = vr::g_ms[k];
            if (bytes) *bytes = vr::g_bytes[k];
            if (launches) *launches = vr::g_launch[k];
            return RAD_OK;
        }
    }
    return RAD_EINVAL;
}

extern "C" const char *rad_last_error(void) { return vr::g_err.c_str(); }

extern "C" const char *rad_build_id(void) { return VETTAM_BUILD_ID; }

extern "C" void rad_default_params(rad_params_t *p)
{
    if (!p) return;
    p->c = 1.0;
    p->a_R = 1.0;
    p->c_v = 1.0;
    p->tol = 1e-10;
    p->eps_R = 1e-2;
    p->eps_P = 0.0;
    p->max_picard = 50;
    p->max_krylov = 20000;
    p->gmres_m = 12;
    p->prec = RAD_FP64;
    p->mode = RAD_PICARD_LINEARISED;
    p->coef_dtype = RAD_F64;
    p->anderson_m = 0;
    p->vel_implicit = 0;
    p->cv_cubic = 0;
    p->krylov_poly = 1;
    for (int f = 0; f < 6; ++f) p->F_inc[f] = 0.0;
    p->eps_N = 0.0;
    p->energy_fix = 0;
    p->max_refine = 0;
    for (int f = 0; f < 6; ++f) p->ghost[f] = nullptr;
}

// ------------------------------------------------------------------ autotune cache

namespace vr {

static std::string cache_file()
{
    const char *d = std::getenv("VETTAM_RAD_CACHE_DIR");
    std::string dir;
    if (d && d[0])
        dir = d;
    else if (const char *h = std::getenv("HOME"))
        dir = std::string(h) + "/.cache/vettam_rad";
    else
        return "";
    // create the directory levels that are missing (no shell involved)
    for (size_t pos = 1; pos <= dir.size(); ++pos)
        if (pos == dir.size() || dir[pos] == '/') (void)mkdir(dir.substr(0, pos).c_str(), 0755);
    return dir + "/autotune.txt";
}

bool cache_get(const std::string &key, std::string &value)
{
    const std::string path = cache_file();
    if (path.empty()) return false;
    std::ifstream in(path);
    std::string line;
    bool found = false;
    while (std::getline(in, line)) {
        const size_t t = line.find('\t');
        if (t == std::string::npos || line.compare(0, t, key) != 0 || t != key.size()) continue;
        value = line.substr(t + 1);
        found = true;
    }
    return found;
}

void cache_put(const std::string &key, const std::string &value)
{
    const std::string path = cache_file();
    if (path.empty()) return;
    std::ofstream out(path, std::ios::app);
    if (out) out << key << "\t" << value << "\n";
}

std::string device_tag()
{
    int dev = 0, cus = 0;
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        cus = prop.multiProcessorCount;
    }
    // the build id keeps tuned entries of one build from steering another
    return arch + "|cu" + std::to_string(cus) + "|" + VETTAM_BUILD_ID;
}

}  // namespace vr
