// Time update (Section 2.2): Verlet scheme, eqs. sphu1, sphr1, sphrho1,
// with the Euler reset of eqs. sphu2, sphr2, sphrho2 every N_s steps (and at
// the first step, which has no previous level).  FP64 accumulators for
// positions and velocities in both precisions; the mixed path keeps the
// density as FP32 (rho - rho0), updated in FP64 and rounded once.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "common.h"

namespace wcsph {

struct IntegrateArgs {
    int64_t n;
    double *x, *y, *z;
    const double *ux, *uy, *uz;
    double *uxm, *uym, *uzm;  // in: u at t - dt; out: u at t + dt
    const void *rho;
    void *rhom;               // in: rho at t - dt; out: rho at t + dt
    const uint32_t *id;
    const void *rates;        // ax, ay, az, drho (n each)
    DevScalars *sc;
    double dt_arg, cfl;
    int euler;
};

template <bool kMixed>
__global__ void k_integrate(IntegrateArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // dt: the caller's, or Cr times the bound reduced by the interaction
    const double dt = a.dt_arg > 0.0 ? a.dt_arg
                                     : a.cfl * __longlong_as_double((long long)a.sc->dt_min_bits);
    if (i == 0) {
        const double cflb = a.cfl * __longlong_as_double((long long)a.sc->dt_min_bits);
        a.sc->dt_cfl = cflb;
        a.sc->dt_last = dt;
        a.sc->time += dt;
        a.sc->steps += 1;
        if (dt > cflb) a.sc->dt_cfl_violation = 1u;
    }
    if (i >= a.n) return;
    const int64_t n = a.n;
    double ax, ay, az, dr;
    if constexpr (kMixed) {
        const float *r = static_cast<const float *>(a.rates);
        ax = r[i];
        ay = r[n + i];
        az = r[2 * n + i];
        dr = r[3 * n + i];
    } else {
        const double *r = static_cast<const double *>(a.rates);
        ax = r[i];
        ay = r[n + i];
        az = r[2 * n + i];
        dr = r[3 * n + i];
    }
    const double w = a.euler ? dt : 2.0 * dt;
    if constexpr (kMixed) {
        const double cur = (double)static_cast<const float *>(a.rho)[i];
        float *pm = static_cast<float *>(a.rhom);
        const double base = a.euler ? cur : (double)pm[i];
        pm[i] = (float)(base + w * dr);
    } else {
        const double cur = static_cast<const double *>(a.rho)[i];
        double *pm = static_cast<double *>(a.rhom);
        const double base = a.euler ? cur : pm[i];
        pm[i] = base + w * dr;
    }
    const double ux = a.ux[i], uy = a.uy[i], uz = a.uz[i];
    if ((a.id[i] >> 31) != 0) {  // boundary: does not move
        a.uxm[i] = ux;
        a.uym[i] = uy;
        a.uzm[i] = uz;
        return;
    }
    const double hdt2 = 0.5 * dt * dt;
    const double bx = a.euler ? ux : a.uxm[i];
    const double by = a.euler ? uy : a.uym[i];
    const double bz = a.euler ? uz : a.uzm[i];
    a.x[i] = a.x[i] + dt * ux + hdt2 * ax;
    a.y[i] = a.y[i] + dt * uy + hdt2 * ay;
    a.z[i] = a.z[i] + dt * uz + hdt2 * az;
    a.uxm[i] = bx + w * ax;
    a.uym[i] = by + w * ay;
    a.uzm[i] = bz + w * az;
}

int launch_integrate(const sph_params &p, sph_state &s, const Ws &w, double dt, int64_t step,
                     hipStream_t st) {
    IntegrateArgs a;
    a.n = s.n;
    a.x = s.x;
    a.y = s.y;
    a.z = s.z;
    a.ux = s.ux;
    a.uy = s.uy;
    a.uz = s.uz;
    a.uxm = s.uxm;
    a.uym = s.uym;
    a.uzm = s.uzm;
    a.rho = s.rho;
    a.rhom = s.rhom;
    a.id = s.id;
    a.rates = w.base + w.L.rates;
    a.sc = w.scalars();
    a.dt_arg = dt;
    a.cfl = p.cfl;
    a.euler = (step == 0) || (p.verlet_ns > 0 && step % p.verlet_ns == 0);
    const int blocks = (int)((s.n + 255) / 256);
    if (p.precision == SPH_MIXED)
        hipLaunchKernelGGL(k_integrate<true>, dim3(blocks), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_integrate<false>, dim3(blocks), dim3(256), 0, st, a);
    if (int rc = launch_check("integrate")) return rc;
    // the new level was written over the previous one: rotate the pointers
    auto swp = [](auto &u, auto &v) { auto t = u; u = v; v = t; };
    swp(s.ux, s.uxm);
    swp(s.uy, s.uym);
    swp(s.uz, s.uzm);
    swp(s.rho, s.rhom);
    return 0;
}

// --------------------------------------------------- density conversion

__global__ void k_set_density(const double *__restrict__ src, void *dst, int64_t n, double rho0,
                              int mixed) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (mixed)
        static_cast<float *>(dst)[i] = (float)(src[i] - rho0);
    else
        static_cast<double *>(dst)[i] = src[i];
}

__global__ void k_get_density(const void *src, double *__restrict__ dst, int64_t n, double rho0,
                              int mixed) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (mixed)
        dst[i] = rho0 + (double)static_cast<const float *>(src)[i];
    else
        dst[i] = static_cast<const double *>(src)[i];
}

int launch_set_density(const sph_params &p, sph_state &s, const double *rho, int which,
                       hipStream_t st) {
    void *dst = which == 0 ? s.rho : s.rhom;
    const int blocks = (int)((s.n + 255) / 256);
    hipLaunchKernelGGL(k_set_density, dim3(blocks), dim3(256), 0, st, rho, dst, s.n, p.rho0,
                       (int)(p.precision == SPH_MIXED));
    return launch_check("set density");
}

int launch_get_density(const sph_params &p, const sph_state &s, double *rho, int which,
                       hipStream_t st) {
    const void *src = which == 0 ? s.rho : s.rhom;
    const int blocks = (int)((s.n + 255) / 256);
    hipLaunchKernelGGL(k_get_density, dim3(blocks), dim3(256), 0, st, src, rho, s.n, p.rho0,
                       (int)(p.precision == SPH_MIXED));
    return launch_check("get density");
}

// ------------------------------------------------------ workspace scalars

__global__ void k_ws_init(DevScalars *sc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        sc->dt_min_bits = 0x7ff0000000000000ull;
        sc->dt_cfl = 0.0;
        sc->dt_last = 0.0;
        sc->time = 0.0;
        sc->steps = 0;
        sc->nchunks = 0;
        sc->dt_cfl_violation = 0;
        sc->pairs[0] = sc->pairs[1] = sc->pairs[2] = 0;
        sc->work = 0;
    }
}

int launch_ws_init(const Ws &w, hipStream_t st) {
    hipLaunchKernelGGL(k_ws_init, dim3(1), dim3(64), 0, st, w.scalars());
    return launch_check("workspace init");
}

}  // namespace wcsph
