// FP64 global diagnostics and Shepard-filtered probe pressures (eq. sphpa).
// Sums use a fixed assignment of particles to threads and fixed reduction
// trees, so they are bit-reproducible for a given particle order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "common.h"

namespace wcsph {

enum {
    F_MASS = 0, F_PX, F_PY, F_PZ, F_EKIN, F_EPOT, F_EINT, F_UMAX, F_NFLUID, F_NONFIN, F_OUTSIDE,
    F_DENS, F_FRONT, F_COUNT
};
static_assert(F_COUNT <= kDiagFields, "diagnostic fields");

__device__ __forceinline__ bool is_max_field(int f) {
    return f == F_UMAX || f == F_DENS || f == F_FRONT;
}

struct DiagArgs {
    const double *x, *y, *z, *ux, *uy, *uz;
    const void *rho;
    const uint32_t *id;
    const uint32_t *cell_start;
    int mixed;
    Insts I;
    int bpi;       // partial-sum blocks per instance
    double *part;  // ninst x bpi x kDiagFields
};

__device__ __forceinline__ int diag_axis(double v, double o, double cs, int n, bool *out) {
    double f = floor((v - o) / cs);
    if (!(f >= 0.0)) {
        *out = true;
        return 0;
    }
    if (f > (double)(n - 1)) {
        *out = true;
        return n - 1;
    }
    return (int)f;
}

__device__ __forceinline__ double density_at(const DiagArgs &a, const Inst &ip, int64_t i) {
    return a.mixed ? ip.rho0 + (double)static_cast<const float *>(a.rho)[i]
                   : static_cast<const double *>(a.rho)[i];
}

// Instance blockIdx.y, its particles [start of its first cell,
// end of its last cell) of the current (cell) order, split over
// bpi blocks with a fixed stride: fixed summation order.
__global__ __launch_bounds__(kDiagThreads) void k_diag_partial(DiagArgs a) {
    __shared__ double red[F_COUNT * (kDiagThreads / kWave)];
    const int k = blockIdx.y;
    const Inst ip = a.I.get(k);
    const int64_t ncell = (int64_t)ip.nx * ip.ny * ip.nz;
    const int64_t lo = a.cell_start[2 * ip.cell_base];
    const int64_t hi = a.cell_start[2 * (ip.cell_base + ncell)];
    const double B = ip.B, rho0 = ip.rho0, gamma = ip.gamma, mass = ip.mass;
    double acc[F_COUNT];
    for (int f = 0; f < F_COUNT; ++f) acc[f] = 0.0;
    acc[F_FRONT] = -INFINITY;
    const int64_t stride = (int64_t)a.bpi * blockDim.x;
    const double gm1 = gamma - 1.0;
    // a fluid particle within 2h of (x, y, z), other than i, at j?
    auto near = [&](int64_t j, int64_t i, double x, double y, double z) {
        if (j < lo || j >= hi || j == i || (a.id[j] >> 31) != 0) return false;
        const double dx = a.x[j] - x, dy_ = a.y[j] - y, dz_ = a.z[j] - z;
        return (dx * dx + dy_ * dy_) + dz_ * dz_ < ip.r2max;
    };
    // the block's rounds are uniform (every lane takes part in the wave
    // operations of the surge-front test)
    for (int64_t b0 = lo + (int64_t)blockIdx.x * blockDim.x; b0 < hi; b0 += stride) {
        const int64_t i = b0 + threadIdx.x;
        const bool live = i < hi;
        const int64_t ii = live ? i : lo;
        const double x = a.x[ii], y = a.y[ii], z = a.z[ii];
        const double ux = a.ux[ii], uy = a.uy[ii], uz = a.uz[ii];
        const double rho = density_at(a, ip, ii);
        const bool bnd = (a.id[ii] >> 31) != 0;
        const bool fluid = live && !bnd;
        int cx = 0, cy = 0, cz = 0;
        if (live) {
            acc[F_MASS] += mass;
            const double rr = rho / rho0;
            acc[F_EINT] += mass * (B / rho0) * (pow(rr, gm1) / gm1 + 1.0 / rr - gamma / gm1);
            const double vals[7] = {x, y, z, ux, uy, uz, rho};
            for (int q = 0; q < 7; ++q)
                if (!isfinite(vals[q])) acc[F_NONFIN] += 1.0;
            bool out = false;
            cx = diag_axis(x, ip.ox, ip.cs, ip.nx, &out);
            cy = diag_axis(y, ip.oy, ip.cs, ip.ny, &out);
            cz = diag_axis(z, ip.oz, ip.cs, ip.nz, &out);
            if (out) acc[F_OUTSIDE] += 1.0;
            acc[F_DENS] = fmax(acc[F_DENS], fabs(rho - rho0) / rho0);
        }
        if (fluid) {
            acc[F_NFLUID] += 1.0;
            acc[F_PX] += mass * ux;
            acc[F_PY] += mass * uy;
            acc[F_PZ] += mass * uz;
            const double u2 = (ux * ux + uy * uy) + uz * uz;
            acc[F_EKIN] += 0.5 * mass * u2;
            acc[F_EPOT] -= mass * ((ip.gx * x + ip.gy * y) + ip.gz * z);
            acc[F_UMAX] = fmax(acc[F_UMAX], sqrt(u2));
        }
        // surge front: the largest x of a fluid particle with at least one
        // fluid neighbour.  The particles next to i in cell order (usually
        // within 2h) settle most; the 27 cells are searched only for a
        // particle that could still raise the maximum, i.e. beyond every
        // particle of its wave settled so far.
        const bool quick = fluid && (near(i + 1, i, x, y, z) || near(i - 1, i, x, y, z));
        double mq = quick ? x : -INFINITY;
        for (int off = kWave / 2; off > 0; off >>= 1) mq = fmax(mq, __shfl_xor(mq, off, kWave));
        if (quick) acc[F_FRONT] = fmax(acc[F_FRONT], x);
        if (fluid && !quick && x > fmax(mq, acc[F_FRONT])) {
            bool found = false;
            for (int dz = -1; dz <= 1 && !found; ++dz)
                for (int dy = -1; dy <= 1 && !found; ++dy) {
                    const int czn = cz + dz, cyn = cy + dy;
                    if (czn < 0 || czn >= ip.nz || cyn < 0 || cyn >= ip.ny) continue;
                    // the fluid half of the stencil row
                    const uint32_t hb = half_row_key(ip, czn * ip.ny + cyn, 0);
                    const int xl = cx > 0 ? cx - 1 : 0, xh = cx + 1 < ip.nx ? cx + 1 : ip.nx - 1;
                    const uint32_t js = a.cell_start[hb + xl], je = a.cell_start[hb + xh + 1];
                    for (uint32_t j = js; j < je && !found; ++j) found = near(j, i, x, y, z);
                }
            if (found) acc[F_FRONT] = x;
        }
    }
    // fixed reduction trees: shuffles within each wave, then the waves in
    // order (one barrier)
    double *part = a.part + ((size_t)k * a.bpi + blockIdx.x) * kDiagFields;
    constexpr int kWaves = kDiagThreads / kWave;
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
#pragma unroll
    for (int f = 0; f < F_COUNT; ++f) {
        double v = acc[f];
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const double o = __shfl_xor(v, off, kWave);
            v = is_max_field(f) ? fmax(v, o) : v + o;
        }
        if (lane == 0) red[f * kWaves + w] = v;
    }
    __syncthreads();
    if (threadIdx.x < F_COUNT) {
        const int f = threadIdx.x;
        double v = red[f * kWaves];
        for (int q = 1; q < kWaves; ++q)
            v = is_max_field(f) ? fmax(v, red[f * kWaves + q]) : v + red[f * kWaves + q];
        part[f] = v;
    }
}

// One block per instance: its bpi partials -> kDiagFields results.
__global__ __launch_bounds__(kDiagThreads) void k_diag_final(const double *__restrict__ part_all,
                                                             int nparts, double *__restrict__ res_all) {
    constexpr int kWaves = kDiagThreads / kWave;
    __shared__ double red[F_COUNT * kWaves];
    const double *part = part_all + (size_t)blockIdx.x * nparts * kDiagFields;
    double *res = res_all + (size_t)blockIdx.x * kDiagFields;
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    for (int f = 0; f < F_COUNT; ++f) {
        const bool mx = is_max_field(f);
        double v = mx ? -INFINITY : 0.0;
        for (int b = threadIdx.x; b < nparts; b += kDiagThreads) {
            const double o = part[b * kDiagFields + f];
            v = mx ? fmax(v, o) : v + o;
        }
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const double o = __shfl_xor(v, off, kWave);
            v = mx ? fmax(v, o) : v + o;
        }
        if (lane == 0) red[f * kWaves + w] = v;
    }
    __syncthreads();
    if (threadIdx.x < F_COUNT) {
        const int f = threadIdx.x;
        double v = red[f * kWaves];
        for (int q = 1; q < kWaves; ++q)
            v = is_max_field(f) ? fmax(v, red[f * kWaves + q]) : v + red[f * kWaves + q];
        res[f] = v;
    }
}

// Wendland C2 kernel value in FP64 (eq. sphw, 3D constant 21/(16 pi h^3)).
__device__ __forceinline__ double wendland(double q, double wd) {
    if (q >= 2.0) return 0.0;
    const double t = 1.0 - 0.5 * q;
    const double t2 = t * t;
    return wd * t2 * t2 * (2.0 * q + 1.0);
}

// One workgroup per probe point: P_a = sum P_b W_ab / sum W_ab over fluid b.
__global__ __launch_bounds__(kDiagThreads) void k_probes(DiagArgs a, const double *__restrict__ pts,
                                                         double *__restrict__ out) {
    __shared__ double rn[kDiagThreads], rd[kDiagThreads];
    const Inst ip = a.I.get(0);
    const double h = ip.h;
    const int pa = blockIdx.x;
    const double px = pts[3 * pa], py = pts[3 * pa + 1], pz = pts[3 * pa + 2];
    bool dummy = false;
    const int cx = diag_axis(px, ip.ox, ip.cs, ip.nx, &dummy);
    const int cy = diag_axis(py, ip.oy, ip.cs, ip.ny, &dummy);
    const int cz = diag_axis(pz, ip.oz, ip.cs, ip.nz, &dummy);
    const double wd = 21.0 / (16.0 * M_PI * h * h * h);
    double num = 0.0, den = 0.0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy) {
            const int czn = cz + dz, cyn = cy + dy;
            if (czn < 0 || czn >= ip.nz || cyn < 0 || cyn >= ip.ny) continue;
            // the fluid half of the stencil row
            const uint32_t hb = half_row_key(ip, czn * ip.ny + cyn, 0);
            const int xl = cx > 0 ? cx - 1 : 0, xh = cx + 1 < ip.nx ? cx + 1 : ip.nx - 1;
            const uint32_t js = a.cell_start[hb + xl], je = a.cell_start[hb + xh + 1];
            for (uint32_t j = js + threadIdx.x; j < je; j += kDiagThreads) {
                if ((a.id[j] >> 31) != 0) continue;
                const double dx = a.x[j] - px, dy_ = a.y[j] - py, dz_ = a.z[j] - pz;
                const double r2 = (dx * dx + dy_ * dy_) + dz_ * dz_;
                if (!(r2 < ip.r2max)) continue;
                const double w = wendland(sqrt(r2) / h, wd);
                const double rho = density_at(a, ip, j);
                const double P = ip.B * (pow(rho / ip.rho0, ip.gamma) - 1.0);
                num += P * w;
                den += w;
            }
        }
    rn[threadIdx.x] = num;
    rd[threadIdx.x] = den;
    __syncthreads();
    for (int off = kDiagThreads / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            rn[threadIdx.x] += rn[threadIdx.x + off];
            rd[threadIdx.x] += rd[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[pa] = rd[0] > 0.0 ? rn[0] / rd[0] : 0.0;
}

int diag_blocks(int ninst) { return ninst == 1 ? kDiagBlocks : kDiagBlocksBatch; }

static DiagArgs diag_args(const Problem &P, const sph_state &s, const Ws &w) {
    DiagArgs a;
    a.x = s.x;
    a.y = s.y;
    a.z = s.z;
    a.ux = s.ux;
    a.uy = s.uy;
    a.uz = s.uz;
    a.rho = s.rho;
    a.id = s.id;
    a.cell_start = w.cell_start();
    a.mixed = P.precision == SPH_MIXED;
    a.I = insts_of(P, w);
    a.bpi = diag_blocks((int)P.host.size());
    a.part = w.diag_part();
    return a;
}

int launch_probes(const Problem &P, const sph_state &s, const Ws &w, const double *probes,
                  int32_t np, double *pout, hipStream_t st) {
    if (np <= 0) return SPH_OK;
    const DiagArgs a = diag_args(P, s, w);
    double *pts = a.part + (size_t)P.host.size() * a.bpi * kDiagFields +
                  (size_t)P.host.size() * kDiagFields;
    if (int rc = hip_check(hipMemcpyAsync(pts, probes, sizeof(double) * 3 * np,
                                          hipMemcpyHostToDevice, st),
                           "probe upload"))
        return rc;
    hipLaunchKernelGGL(k_probes, dim3(np), dim3(kDiagThreads), 0, st, a, pts, pout);
    return launch_check("probes");
}

// out: ninst results (instance order); probes: instance 0 only.
int launch_diag(const Problem &P, const sph_state &s, const Ws &w, const double *probes,
                int32_t np, sph_diag *out, double *probe_p, hipStream_t st) {
    const int ninst = (int)P.host.size();
    const DiagArgs a = diag_args(P, s, w);
    double *res = a.part + (size_t)ninst * a.bpi * kDiagFields;
    double *pts = res + (size_t)ninst * kDiagFields;
    double *pout = pts + 3 * kMaxProbes;
    hipLaunchKernelGGL(k_diag_partial, dim3(a.bpi, ninst), dim3(kDiagThreads), 0, st, a);
    hipLaunchKernelGGL(k_diag_final, dim3(ninst), dim3(kDiagThreads), 0, st, a.part, a.bpi, res);
    if (int rc = launch_check("diagnostics")) return rc;
    if (int rc = launch_probes(P, s, w, probes, np, pout, st)) return rc;
    std::vector<double> host((size_t)ninst * kDiagFields);
    std::vector<InstState> ist(ninst);
    DevScalars sc;
    if (int rc = hip_check(hipMemcpyAsync(host.data(), res, sizeof(double) * host.size(),
                                          hipMemcpyDeviceToHost, st),
                           "diagnostics download"))
        return rc;
    if (int rc = hip_check(hipMemcpyAsync(ist.data(), w.inst_state(), sizeof(InstState) * ninst,
                                          hipMemcpyDeviceToHost, st),
                           "clock download"))
        return rc;
    if (int rc = hip_check(hipMemcpyAsync(&sc, w.scalars(), sizeof(sc), hipMemcpyDeviceToHost, st),
                           "scalars download"))
        return rc;
    if (np > 0) {
        if (int rc = hip_check(hipMemcpyAsync(probe_p, pout, sizeof(double) * np,
                                              hipMemcpyDeviceToHost, st),
                               "probe download"))
            return rc;
    }
    if (int rc = hip_check(hipStreamSynchronize(st), "diagnostics sync")) return rc;
    for (int k = 0; k < ninst; ++k) {
        const double *hv = host.data() + (size_t)k * kDiagFields;
        const Inst &ip = P.host[k];
        sph_diag *o = out + k;
        std::memset(o, 0, sizeof(*o));
        o->mass = hv[F_MASS];
        o->mom[0] = hv[F_PX];
        o->mom[1] = hv[F_PY];
        o->mom[2] = hv[F_PZ];
        o->e_kin = hv[F_EKIN];
        o->e_pot = hv[F_EPOT];
        o->e_int = hv[F_EINT];
        o->umax = hv[F_UMAX];
        o->x_front = hv[F_FRONT];
        o->dt_cfl = ist[k].dt_cfl;
        o->dt_last = ist[k].dt_last;
        o->time = ist[k].time;
        o->n = (int64_t)ip.pend - (int64_t)ip.pstart;
        o->n_fluid = (int64_t)hv[F_NFLUID];
        o->n_outside = (int64_t)hv[F_OUTSIDE];
        o->n_nonfinite = (int64_t)hv[F_NONFIN];
        o->steps = sc.steps;
        // the chunk records hold FF + FB (fluid targets) and BF (boundary
        // targets); FB equals BF (the neighbour relation is symmetric)
        o->pairs_ff = (int64_t)sc.pairs[0] - (int64_t)sc.pairs[2];
        o->pairs_fb = (int64_t)sc.pairs[2];
        o->pairs_bf = (int64_t)sc.pairs[2];
        uint32_t flags = 0;
        if (o->n_nonfinite > 0) flags |= SPH_FLAG_NONFINITE;
        if (o->n_outside > 0) flags |= SPH_FLAG_OUTSIDE;
        if (hv[F_DENS] > 0.1) flags |= SPH_FLAG_DENSITY;
        if (sc.dt_cfl_violation) flags |= SPH_FLAG_DT_CFL;
        o->flags = flags;
    }
    return 0;
}

}  // namespace wcsph
