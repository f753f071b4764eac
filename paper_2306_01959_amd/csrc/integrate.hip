// Time update (Section 2.2): Verlet scheme, eqs. sphu1, sphr1, sphrho1,
// with the Euler reset of eqs. sphu2, sphr2, sphrho2 every N_s steps (and at
// the first step, which has no previous level).  FP64 accumulators for
// positions and velocities in both precisions; the mixed path keeps the
// density as FP32 (rho - rho0), updated in FP64 and rounded once.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "common.h"
#include "update.h"

namespace wcsph {

struct IntegrateArgs {
    int64_t n;
    StateArrays state;
    const void *rates;  // ax, ay, az, drho (n each)
    Insts I;
    DevScalars *sc;
    InstState *ist;
    double dt_arg;
    long long step;
    uint32_t *hist;  // digit counts per sort tile (digit-major), or null
    int hist_shift;
    int ntiles;
};

// dt of the instance for this step: the caller's, or Cr times the bound
// reduced by this step's interaction (eq. sphdt)
__device__ __forceinline__ double step_dt(const IntegrateArgs &a, const Inst &ip, int k) {
    const double b = __longlong_as_double((long long)a.ist[k].dt_min_bits);
    return a.dt_arg > 0.0 ? a.dt_arg : ip.cfl * b;
}

// Block b updates the particles of sort tile b (kItems per thread, block-
// strided) and, with a.hist, counts the digits of the keys it writes: the
// histogram of the next sort's first pass.  Blocks of kUpdateThreads, so that
// a small tile is one particle per thread (a thread's particles are updated
// one after the other).
constexpr int kUpdateThreads = 1024;
template <bool kMixed, int kItems>
__global__ __launch_bounds__(kUpdateThreads) void k_integrate(IntegrateArgs a) {
    __shared__ uint32_t h[kRadix];
    const int tid = threadIdx.x;
    if (blockIdx.x == 0) {
        // per-instance clock
        for (int k = tid; k < a.I.n; k += blockDim.x) {
            const Inst ip = a.I.get(k);
            const double b = __longlong_as_double((long long)a.ist[k].dt_min_bits);
            const double dt = step_dt(a, ip, k);
            a.ist[k].dt_cfl = ip.cfl * b;
            a.ist[k].dt_last = dt;
            a.ist[k].time += dt;
            if (dt > ip.cfl * b) a.sc->dt_cfl_violation = 1u;
        }
        if (tid == 0) a.sc->steps += 1;
    }
    if (a.hist) {
        for (int d = tid; d < kRadix; d += kUpdateThreads) h[d] = 0;
        __syncthreads();
    }
    const int64_t n = a.n;
    const int tile = tile_of_block(blockIdx.x, a.ntiles);
    const int64_t base = (int64_t)tile * kUpdateThreads * kItems;
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int64_t i = base + (int64_t)it * kUpdateThreads + tid;
        const bool ok = i < n;
        uint32_t key = 0;
        if (ok) {
            const int k = a.I.of_id(a.state.id[i] & 0x7fffffffu);
            const Inst ip = a.I.get(k);
            const double dt = step_dt(a, ip, k);
            const bool euler = a.step == 0 || (ip.verlet_ns > 0 && a.step % ip.verlet_ns == 0);
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
            key = advance<kMixed, true>(a.state, ip, i, dt, euler, ax, ay, az, dr);
        }
        if (a.hist) tile_hist_add(h, key, ok, a.hist_shift);
    }
    if (a.hist) {
        __syncthreads();
        for (int d = tid; d < kRadix; d += kUpdateThreads)
            a.hist[(int64_t)d * a.ntiles + tile] = h[d];
    }
}

static void rotate_levels(sph_state &s) {
    // the new level was written over the previous one
    auto swp = [](auto &u, auto &v) { auto t = u; u = v; v = t; };
    swp(s.ux, s.uxm);
    swp(s.uy, s.uym);
    swp(s.uz, s.uzm);
    swp(s.rho, s.rhom);
}

int launch_integrate(const Problem &P, sph_state &s, const Ws &w, double dt, int64_t step,
                     hipStream_t st, int hist_shift) {
    IntegrateArgs a;
    a.n = s.n;
    a.state = StateArrays{s.x,   s.y,   s.z,   s.ux,  s.uy,   s.uz,  s.uxm,
                          s.uym, s.uzm, s.rho, s.rhom, s.id, w.keys_next(),
                          &w.scalars()->walls_move, s.rho_alt, s.rhom_alt};
    a.rates = w.base + w.L.rates;
    a.I = insts_of(P, w);
    a.sc = w.scalars();
    a.ist = w.inst_state();
    a.dt_arg = dt;
    a.step = step;
    a.hist = hist_shift >= 0 ? w.hist() : nullptr;
    a.hist_shift = hist_shift;
    a.ntiles = (int)w.L.ntiles;
    // one block per sort tile (the tiling of the sort's histogram pass)
    constexpr int kSmall = kSortThreads * kSortItemsSmall / kUpdateThreads;
    constexpr int kLarge = kSortThreads * kSortItemsLarge / kUpdateThreads;
    static_assert(kSmall * kUpdateThreads == kSortThreads * kSortItemsSmall &&
                      kLarge * kUpdateThreads == kSortThreads * kSortItemsLarge,
                  "update blocks cover whole sort tiles");
    const bool small = sort_tile(s.n) == (int64_t)kSortThreads * kSortItemsSmall;
    const dim3 grid((unsigned)w.L.ntiles), block(kUpdateThreads);
    if (P.precision == SPH_MIXED) {
        if (small)
            hipLaunchKernelGGL((k_integrate<true, kSmall>), grid, block, 0, st, a);
        else
            hipLaunchKernelGGL((k_integrate<true, kLarge>), grid, block, 0, st, a);
    } else {
        if (small)
            hipLaunchKernelGGL((k_integrate<false, kSmall>), grid, block, 0, st, a);
        else
            hipLaunchKernelGGL((k_integrate<false, kLarge>), grid, block, 0, st, a);
    }
    if (int rc = launch_check("integrate")) return rc;
    rotate_levels(s);
    return 0;
}

// The fused interaction advanced the state in place: rotate the levels.
void after_fused_step(sph_state &s) { rotate_levels(s); }

// ------------------------------------------------ two-stage symplectic step
//
// Predictor (rates at t, in the workspace): the level at t is kept in
// (um, rhom); r* = r + dt/2 u, u* = u + dt/2 a (fluid), rho* = rho + dt/2 drho.
// Corrector (rates at t*): u' = u(t) + dt a* (fluid), r' = r* + dt/2 u',
// rho' = rho(t) + dt drho*.  Boundary particles keep u and move with it.  The
// predictor fixes each instance's dt (the caller's, or Cr x the bound of the
// rates at t) and the corrector reuses it; no level rotation.
struct SymArgs {
    int64_t n;
    double *x, *y, *z, *ux, *uy, *uz, *uxm, *uym, *uzm;
    void *rho, *rhom;
    const uint32_t *id;
    const void *rates;  // ax, ay, az, drho (n each)
    Insts I;
    DevScalars *sc;
    InstState *ist;
    double dt_arg;
};

template <bool kMixed>
__device__ __forceinline__ void sym_rates(const SymArgs &a, int64_t i, double &ax, double &ay,
                                          double &az, double &dr) {
    const int64_t n = a.n;
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
}

template <bool kMixed>
__global__ __launch_bounds__(256) void k_sym_predict(SymArgs a) {
    if (blockIdx.x == 0) {
        for (int k = threadIdx.x; k < a.I.n; k += blockDim.x) {
            const Inst ip = a.I.get(k);
            const double b = __longlong_as_double((long long)a.ist[k].dt_min_bits);
            const double dt = a.dt_arg > 0.0 ? a.dt_arg : ip.cfl * b;
            a.ist[k].dt_cfl = ip.cfl * b;
            a.ist[k].dt_last = dt;
            if (dt > ip.cfl * b) a.sc->dt_cfl_violation = 1u;
        }
    }
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const uint32_t id = a.id[i];
    const int k = a.I.of_id(id & 0x7fffffffu);
    const Inst ip = a.I.get(k);
    const double b = __longlong_as_double((long long)a.ist[k].dt_min_bits);
    const double h2 = 0.5 * (a.dt_arg > 0.0 ? a.dt_arg : ip.cfl * b);
    double ax, ay, az, dr;
    sym_rates<kMixed>(a, i, ax, ay, az, dr);
    if constexpr (kMixed) {
        float *rho = static_cast<float *>(a.rho);
        const float cur = rho[i];
        static_cast<float *>(a.rhom)[i] = cur;
        rho[i] = (float)((double)cur + h2 * dr);
    } else {
        double *rho = static_cast<double *>(a.rho);
        const double cur = rho[i];
        static_cast<double *>(a.rhom)[i] = cur;
        rho[i] = cur + h2 * dr;
    }
    const double ux = a.ux[i], uy = a.uy[i], uz = a.uz[i];
    a.uxm[i] = ux;
    a.uym[i] = uy;
    a.uzm[i] = uz;
    a.x[i] = a.x[i] + h2 * ux;
    a.y[i] = a.y[i] + h2 * uy;
    a.z[i] = a.z[i] + h2 * uz;
    if ((id >> 31) == 0) {
        a.ux[i] = ux + h2 * ax;
        a.uy[i] = uy + h2 * ay;
        a.uz[i] = uz + h2 * az;
    }
}

template <bool kMixed>
__global__ __launch_bounds__(256) void k_sym_correct(SymArgs a) {
    if (blockIdx.x == 0) {
        for (int k = threadIdx.x; k < a.I.n; k += blockDim.x) a.ist[k].time += a.ist[k].dt_last;
        if (threadIdx.x == 0) a.sc->steps += 1;
    }
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const uint32_t id = a.id[i];
    const int k = a.I.of_id(id & 0x7fffffffu);
    const double dt = a.ist[k].dt_last;
    const double h2 = 0.5 * dt;
    double ax, ay, az, dr;
    sym_rates<kMixed>(a, i, ax, ay, az, dr);
    if constexpr (kMixed) {
        const float base = static_cast<const float *>(a.rhom)[i];
        static_cast<float *>(a.rho)[i] = (float)((double)base + dt * dr);
    } else {
        const double base = static_cast<const double *>(a.rhom)[i];
        static_cast<double *>(a.rho)[i] = base + dt * dr;
    }
    double ux = a.uxm[i], uy = a.uym[i], uz = a.uzm[i];
    if ((id >> 31) == 0) {
        ux += dt * ax;
        uy += dt * ay;
        uz += dt * az;
    }
    a.ux[i] = ux;
    a.uy[i] = uy;
    a.uz[i] = uz;
    a.x[i] = a.x[i] + h2 * ux;
    a.y[i] = a.y[i] + h2 * uy;
    a.z[i] = a.z[i] + h2 * uz;
}

int launch_symplectic(const Problem &P, sph_state &s, const Ws &w, double dt, bool corrector,
                      hipStream_t st) {
    SymArgs a;
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
    a.I = insts_of(P, w);
    a.sc = w.scalars();
    a.ist = w.inst_state();
    a.dt_arg = dt;
    const dim3 grid((unsigned)((s.n + 255) / 256)), block(256);
    const bool mixed = P.precision == SPH_MIXED;
    if (corrector) {
        if (mixed)
            hipLaunchKernelGGL((k_sym_correct<true>), grid, block, 0, st, a);
        else
            hipLaunchKernelGGL((k_sym_correct<false>), grid, block, 0, st, a);
    } else {
        if (mixed)
            hipLaunchKernelGGL((k_sym_predict<true>), grid, block, 0, st, a);
        else
            hipLaunchKernelGGL((k_sym_predict<false>), grid, block, 0, st, a);
    }
    return launch_check(corrector ? "symplectic corrector" : "symplectic predictor");
}

// --------------------------------------------------- density conversion

__global__ void k_set_density(const double *__restrict__ src, void *dst, int64_t n, Insts I,
                              const uint32_t *__restrict__ id, int mixed) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (mixed) {
        const double rho0 = I.get(I.of_id(id[i] & 0x7fffffffu)).rho0;
        static_cast<float *>(dst)[i] = (float)(src[i] - rho0);
    } else {
        static_cast<double *>(dst)[i] = src[i];
    }
}

__global__ void k_get_density(const void *src, double *__restrict__ dst, int64_t n, Insts I,
                              const uint32_t *__restrict__ id, int mixed) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (mixed) {
        const double rho0 = I.get(I.of_id(id[i] & 0x7fffffffu)).rho0;
        dst[i] = rho0 + (double)static_cast<const float *>(src)[i];
    } else {
        dst[i] = static_cast<const double *>(src)[i];
    }
}

int launch_set_density(const Problem &P, sph_state &s, const Ws &w, const double *rho, int which,
                       hipStream_t st) {
    void *dst = which == 0 ? s.rho : s.rhom;
    const int blocks = (int)((s.n + 255) / 256);
    hipLaunchKernelGGL(k_set_density, dim3(blocks), dim3(256), 0, st, rho, dst, s.n,
                       insts_of(P, w), s.id, (int)(P.precision == SPH_MIXED));
    return launch_check("set density");
}

int launch_get_density(const Problem &P, const sph_state &s, const Ws &w, double *rho, int which,
                       hipStream_t st) {
    const void *src = which == 0 ? s.rho : s.rhom;
    const int blocks = (int)((s.n + 255) / 256);
    hipLaunchKernelGGL(k_get_density, dim3(blocks), dim3(256), 0, st, src, rho, s.n,
                       insts_of(P, w), s.id, (int)(P.precision == SPH_MIXED));
    return launch_check("get density");
}

// ------------------------------------------------------ workspace scalars

__global__ void k_ws_init(DevScalars *sc, InstState *ist, int ninst, ImpulseState *imp) {
    const int t = threadIdx.x;
    if (t == 0) {
        imp->t_prev = 0.0;
        imp->has_prev = 0;
        imp->np = 0;
        sc->steps = 0;
        sc->nchunks = 0;
        sc->dt_cfl_violation = 0;
        sc->pairs[0] = sc->pairs[1] = sc->pairs[2] = 0;
        sc->walls_move = 0;
        sc->pad = 0;
    }
    for (int k = t; k < ninst; k += blockDim.x) {
        ist[k].dt_min_bits = 0x7ff0000000000000ull;  // +inf: no bound yet
        ist[k].dt_lag_bits = 0x7ff0000000000000ull;
        ist[k].dt_cfl = 0.0;
        ist[k].dt_last = 0.0;
        ist[k].time = 0.0;
        ist[k].pad = 0.0;
    }
}

int launch_ws_init(const Problem &P, const Ws &w, hipStream_t st) {
    if (P.batch) {
        // the instance table lives in the workspace; the host copy is
        // staged by the runtime, so the caller may free it on return
        if (int rc = hip_check(hipMemcpyAsync(w.inst_tab(), P.host.data(),
                                              sizeof(Inst) * P.host.size(),
                                              hipMemcpyHostToDevice, st),
                               "instance table upload"))
            return rc;
        if (int rc = hip_check(hipStreamSynchronize(st), "instance table upload")) return rc;
    }
    hipLaunchKernelGGL(k_ws_init, dim3(1), dim3(256), 0, st, w.scalars(), w.inst_state(),
                       (int)P.host.size(), w.impulse());
    return launch_check("workspace init");
}

}  // namespace wcsph
