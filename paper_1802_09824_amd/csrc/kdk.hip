// Adaptive Kick-Drift-Kick integration (sec. 3.4) driving the whole force,
// pp_accel (short range) + pp_pm_accel (long range), for a non-expanding
// box: the drift and kick integrals of dt / a^2 and dt / a are the step.
// Step lengths are dt / 2^k with the smallest k in [0, max_level] meeting
// the Gadget-2 criterion dt / 2^k <= sqrt(2 eta eps / |a|) (the paper prints
// it with the square root misplaced); the levels are set from the forces at
// the start of a top step and kept for it.  A top step runs 2^K substeps of
// dt / 2^K (K the deepest level in use): opening half kicks for the
// particles whose step starts at the substep, a drift of every particle, the
// forces at the new positions, closing half kicks for the particles whose
// step ends there.  Only those particles need new forces: the short-range
// force is evaluated for them alone (pp_accel_active: the target blocks
// without such a particle are skipped), from all particles as sources; the
// PM force, one mesh solve for everybody, is evaluated in full.  A particle's
// force is therefore fresh whenever a kick uses it: its closing kick
// follows its own evaluation, and its next opening kick uses that same
// force.
#include <cmath>
#include <new>

#include "photon_pp.h"
#include "pp_internal.h"

namespace pp {
namespace {

constexpr int kMaxKdkLevel = 15;

__global__ void __launch_bounds__(256) levels_kernel(const float* __restrict__ a1,
                                                     const float* __restrict__ a2, int64_t n,
                                                     double dt, double two_eta_eps, int max_level,
                                                     int8_t* __restrict__ level,
                                                     int32_t* __restrict__ hist) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double ax = (double)a1[i] + (a2 ? (double)a2[i] : 0.0);
    const double ay = (double)a1[n + i] + (a2 ? (double)a2[n + i] : 0.0);
    const double az = (double)a1[2 * n + i] + (a2 ? (double)a2[2 * n + i] : 0.0);
    const double amag = sqrt(ax * ax + ay * ay + az * az);
    int k = 0;
    if (amag > 0.0) {
        const double t = sqrt(two_eta_eps / amag);
        double h = dt;
        while (k < max_level && h > t) {
            ++k;
            h = dt / (double)(1 << k);
        }
    }
    level[i] = (int8_t)k;
    atomicAdd(&hist[k], 1);
}

// v += a * (dt / 2^k) / 2 for the particles whose step starts (open) or
// ends (close) at substep s of 2^K.
__global__ void __launch_bounds__(256) kick_kernel(double* __restrict__ vel, const float* __restrict__ a1,
                                                   const float* __restrict__ a2,
                                                   const int8_t* __restrict__ level, int64_t n,
                                                   int K, int s, double dt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int k = level[i];
    const int span = 1 << (K - k);
    if (s % span != 0) return;
    const double f = 0.5 * dt / (double)(1 << k);
    vel[i] += f * ((double)a1[i] + (a2 ? (double)a2[i] : 0.0));
    vel[n + i] += f * ((double)a1[n + i] + (a2 ? (double)a2[n + i] : 0.0));
    vel[2 * n + i] += f * ((double)a1[2 * n + i] + (a2 ? (double)a2[2 * n + i] : 0.0));
}

__global__ void __launch_bounds__(256) drift_kernel(double* __restrict__ pos, const double* __restrict__ vel,
                                                    int64_t n3, double h, double L) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3) return;
    const double x = pos[i] + vel[i] * h;
    pos[i] = x - L * floor(x / L);
}

// Flags the particles whose step ends at substep boundary s of 2^K.
__global__ void __launch_bounds__(256) active_kernel(const int8_t* __restrict__ level, int64_t n, int K,
                                                     int s, uint8_t* __restrict__ active) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    active[i] = (s % (1 << (K - level[i]))) == 0 ? 1 : 0;
}

__global__ void zero_i32_kernel(int32_t* __restrict__ p, int n) {
    const int i = threadIdx.x;
    if (i < n) p[i] = 0;
}

}  // namespace
}  // namespace pp

using namespace pp;

struct pp_kdk {
    pp_box_params p{};
    int64_t n = 0;
    double eta = 0;
    int max_level = 0;
    pp_plan* plan = nullptr;
    pp_pm_plan* pm = nullptr;
    DevBuf acc_pp, acc_pm, level, hist, active;
    bool ready = false;
    pp_kdk_info info{};
    ~pp_kdk() {
        if (plan) pp_plan_destroy(plan);
        if (pm) pp_pm_plan_destroy(pm);
    }
    // active: per-particle flags of the targets that need new short-range
    // forces (null: all); n_active of them
    int forces(const double* pos, const float* mass, hipStream_t s, const uint8_t* act,
               int64_t n_active) {
        if (act)
            PP_TRY(pp_accel_active(plan, pos, mass, n, act, acc_pp.as<float>(), (void*)s));
        else
            PP_TRY(pp_accel(plan, pos, mass, n, acc_pp.as<float>(), (void*)s));
        if (pm) PP_TRY(pp_pm_accel(pm, pos, mass, n, acc_pm.as<float>(), (void*)s));
        info.force_evaluations += 1;
        info.short_range_targets += n_active;
        return PP_OK;
    }
};

extern "C" {

int pp_kdk_create(const pp_box_params* p, int32_t n_mesh, int64_t n, double eta, int32_t max_level,
                  pp_kdk** out) {
    if (!out) return fail(PP_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1) return fail(PP_EINVAL, "n must be >= 1");
    if (!(eta > 0.0) || !std::isfinite(eta)) return fail(PP_EINVAL, "eta must be finite and > 0");
    if (max_level < 0 || max_level > kMaxKdkLevel) return fail(PP_EINVAL, "max_level must be in 0..15");
    if (n_mesh != 0 && n_mesh < 4) return fail(PP_EINVAL, "n_mesh must be 0 (no PM) or >= 4");
    PP_TRY(validate_params(p, true));
    if (!(p->eps > 0.0)) return fail(PP_EINVAL, "the step criterion needs eps > 0");
    pp_kdk* k = new (std::nothrow) pp_kdk;
    if (!k) return fail(PP_ENOMEM, "host allocation failed");
    k->p = *p;
    k->n = n;
    k->eta = eta;
    k->max_level = max_level;
    int rc = pp_plan_create(p, n, &k->plan);
    if (rc == PP_OK && n_mesh > 0) rc = pp_pm_plan_create(p, n_mesh, &k->pm);
    if (rc == PP_OK) rc = k->acc_pp.reserve(sizeof(float) * 3 * n);
    if (rc == PP_OK && k->pm) rc = k->acc_pm.reserve(sizeof(float) * 3 * n);
    if (rc == PP_OK) rc = k->level.reserve(n);
    if (rc == PP_OK) rc = k->active.reserve(n);
    if (rc == PP_OK) rc = k->hist.reserve(sizeof(int32_t) * (kMaxKdkLevel + 1));
    if (rc != PP_OK) {
        delete k;
        return rc;
    }
    *out = k;
    return PP_OK;
}

int pp_kdk_init(pp_kdk* k, const double* pos, const float* mass, void* stream) {
    if (!k || !pos || !mass) return fail(PP_EINVAL, "NULL argument");
    PP_TRY(k->forces(pos, mass, (hipStream_t)stream, nullptr, k->n));
    k->ready = true;
    return PP_OK;
}

int pp_kdk_step(pp_kdk* k, double* pos, double* vel, const float* mass, double dt, void* stream) {
    if (!k || !pos || !vel || !mass) return fail(PP_EINVAL, "NULL argument");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(PP_EINVAL, "dt must be finite and > 0");
    if (!k->ready) return fail(PP_EINVAL, "pp_kdk_init must run first");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = k->n;
    const float* a1 = k->acc_pp.as<float>();
    const float* a2 = k->pm ? k->acc_pm.as<float>() : nullptr;
    int8_t* lev = k->level.as<int8_t>();
    int32_t* hist = k->hist.as<int32_t>();
    hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, s, hist, kMaxKdkLevel + 1);
    hipLaunchKernelGGL(levels_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, a1, a2, n, dt,
                       2.0 * k->eta * k->p.eps, k->max_level, lev, hist);
    PP_HIP(hipGetLastError());
    int32_t h[kMaxKdkLevel + 1];
    PP_HIP(hipMemcpyAsync(h, hist, sizeof(h), hipMemcpyDeviceToHost, s));
    PP_HIP(hipStreamSynchronize(s));
    int K = 0;
    for (int l = 0; l <= kMaxKdkLevel; ++l) {
        k->info.level_count[l] = h[l];
        if (h[l] > 0) K = l;
    }
    k->info.deepest_level = K;
    const int nsub = 1 << K;
    const double hsub = dt / (double)nsub;
    uint8_t* act = k->active.as<uint8_t>();
    for (int sub = 0; sub < nsub; ++sub) {
        hipLaunchKernelGGL(kick_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, vel, a1, a2, lev, n, K,
                           sub, dt);
        hipLaunchKernelGGL(drift_kernel, dim3(blocks_for(3 * n, 256)), dim3(256), 0, s, pos, vel, 3 * n,
                           hsub, k->p.L);
        // the particles whose step ends at sub + 1 (all of them at the last one)
        int64_t n_active = 0;
        for (int l = 0; l <= K; ++l)
            if ((sub + 1) % (1 << (K - l)) == 0) n_active += h[l];
        const bool all = n_active == n;
        if (!all)
            hipLaunchKernelGGL(active_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, lev, n, K, sub + 1,
                               act);
        PP_HIP(hipGetLastError());
        PP_TRY(k->forces(pos, mass, s, all ? nullptr : act, n_active));
        hipLaunchKernelGGL(kick_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, vel, a1, a2, lev, n, K,
                           sub + 1, dt);
        PP_HIP(hipGetLastError());
    }
    k->info.top_steps += 1;
    return PP_OK;
}

int pp_kdk_set_skin(pp_kdk* k, double skin) {
    if (!k) return fail(PP_EINVAL, "NULL argument");
    return pp_plan_set_skin(k->plan, skin);
}

int pp_kdk_get_info(const pp_kdk* k, pp_kdk_info* out) {
    if (!k || !out) return fail(PP_EINVAL, "NULL argument");
    *out = k->info;
    pp_stats st{};
    PP_TRY(pp_plan_stats(k->plan, &st));
    out->list_builds = st.list_builds;
    return PP_OK;
}

int pp_kdk_levels(const pp_kdk* k, int8_t* level, void* stream) {
    if (!k || !level) return fail(PP_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    PP_HIP(hipMemcpyAsync(level, k->level.p, k->n, hipMemcpyDeviceToDevice, s));
    return PP_OK;
}

int pp_kdk_accel(const pp_kdk* k, float* acc, void* stream) {
    if (!k || !acc) return fail(PP_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    PP_HIP(hipMemcpyAsync(acc, k->acc_pp.p, sizeof(float) * 3 * k->n, hipMemcpyDeviceToDevice, s));
    if (k->pm)
        PP_HIP(hipMemcpyAsync(acc + 3 * k->n, k->acc_pm.p, sizeof(float) * 3 * k->n, hipMemcpyDeviceToDevice, s));
    return PP_OK;
}

void pp_kdk_destroy(pp_kdk* k) { delete k; }

}  // extern "C"
