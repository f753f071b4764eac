// FP64 global diagnostics and Shepard-filtered probe pressures (eq. sphpa).
// Sums use a fixed assignment of particles to threads and fixed reduction
// trees, so they are bit-reproducible for a given particle order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

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
    int64_t n;
    const double *x, *y, *z, *ux, *uy, *uz;
    const void *rho;
    const uint32_t *id;
    const uint32_t *cell_start;
    int mixed;
    Grid g;
    double mass, rho0, B, gamma, gx, gy, gz, r2max;
    double *part;  // kDiagBlocks x kDiagFields
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

__device__ __forceinline__ double density_at(const DiagArgs &a, int64_t i) {
    return a.mixed ? a.rho0 + (double)static_cast<const float *>(a.rho)[i]
                   : static_cast<const double *>(a.rho)[i];
}

__global__ __launch_bounds__(kDiagThreads) void k_diag_partial(DiagArgs a) {
    __shared__ double red[kDiagThreads];
    double acc[F_COUNT];
    for (int f = 0; f < F_COUNT; ++f) acc[f] = 0.0;
    acc[F_FRONT] = -INFINITY;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const double gm1 = a.gamma - 1.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        const double x = a.x[i], y = a.y[i], z = a.z[i];
        const double ux = a.ux[i], uy = a.uy[i], uz = a.uz[i];
        const double rho = density_at(a, i);
        const bool bnd = (a.id[i] >> 31) != 0;
        acc[F_MASS] += a.mass;
        const double rr = rho / a.rho0;
        acc[F_EINT] += a.mass * (a.B / a.rho0) * (pow(rr, gm1) / gm1 + 1.0 / rr - a.gamma / gm1);
        const double vals[7] = {x, y, z, ux, uy, uz, rho};
        for (int k = 0; k < 7; ++k)
            if (!isfinite(vals[k])) acc[F_NONFIN] += 1.0;
        bool out = false;
        const int cx = diag_axis(x, a.g.ox, a.g.cs, a.g.nx, &out);
        const int cy = diag_axis(y, a.g.oy, a.g.cs, a.g.ny, &out);
        const int cz = diag_axis(z, a.g.oz, a.g.cs, a.g.nz, &out);
        if (out) acc[F_OUTSIDE] += 1.0;
        acc[F_DENS] = fmax(acc[F_DENS], fabs(rho - a.rho0) / a.rho0);
        if (bnd) continue;
        acc[F_NFLUID] += 1.0;
        acc[F_PX] += a.mass * ux;
        acc[F_PY] += a.mass * uy;
        acc[F_PZ] += a.mass * uz;
        const double u2 = (ux * ux + uy * uy) + uz * uz;
        acc[F_EKIN] += 0.5 * a.mass * u2;
        acc[F_EPOT] -= a.mass * ((a.gx * x + a.gy * y) + a.gz * z);
        acc[F_UMAX] = fmax(acc[F_UMAX], sqrt(u2));
        if (!(x > acc[F_FRONT])) continue;
        // surge front: fluid particle with at least one fluid neighbour
        bool found = false;
        for (int dz = -1; dz <= 1 && !found; ++dz)
            for (int dy = -1; dy <= 1 && !found; ++dy) {
                const int czn = cz + dz, cyn = cy + dy;
                if (czn < 0 || czn >= a.g.nz || cyn < 0 || cyn >= a.g.ny) continue;
                const int64_t rb = lin_cell(0, cyn, czn, a.g.nx, a.g.ny);
                const int xl = cx > 0 ? cx - 1 : 0, xh = cx + 1 < a.g.nx ? cx + 1 : a.g.nx - 1;
                const uint32_t js = a.cell_start[rb + xl], je = a.cell_start[rb + xh + 1];
                for (uint32_t j = js; j < je; ++j) {
                    if ((int64_t)j == i || (a.id[j] >> 31) != 0) continue;
                    const double dx = a.x[j] - x, dy_ = a.y[j] - y, dz_ = a.z[j] - z;
                    if ((dx * dx + dy_ * dy_) + dz_ * dz_ < a.r2max) {
                        found = true;
                        break;
                    }
                }
            }
        if (found) acc[F_FRONT] = x;
    }
    for (int f = 0; f < F_COUNT; ++f) {
        red[threadIdx.x] = acc[f];
        __syncthreads();
        for (int off = kDiagThreads / 2; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off) {
                const double o = red[threadIdx.x + off];
                red[threadIdx.x] = is_max_field(f) ? fmax(red[threadIdx.x], o) : red[threadIdx.x] + o;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) a.part[blockIdx.x * kDiagFields + f] = red[0];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kDiagThreads) void k_diag_final(const double *__restrict__ part,
                                                             int nparts, double *__restrict__ res) {
    __shared__ double red[kDiagThreads];
    for (int f = 0; f < F_COUNT; ++f) {
        const bool mx = is_max_field(f);
        double v = mx ? -INFINITY : 0.0;
        for (int b = threadIdx.x; b < nparts; b += kDiagThreads) {
            const double o = part[b * kDiagFields + f];
            v = mx ? fmax(v, o) : v + o;
        }
        red[threadIdx.x] = v;
        __syncthreads();
        for (int off = kDiagThreads / 2; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off) {
                const double o = red[threadIdx.x + off];
                red[threadIdx.x] = mx ? fmax(red[threadIdx.x], o) : red[threadIdx.x] + o;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) res[f] = red[0];
        __syncthreads();
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
                                                         double h, double *__restrict__ out) {
    __shared__ double rn[kDiagThreads], rd[kDiagThreads];
    const int pa = blockIdx.x;
    const double px = pts[3 * pa], py = pts[3 * pa + 1], pz = pts[3 * pa + 2];
    bool dummy = false;
    const int cx = diag_axis(px, a.g.ox, a.g.cs, a.g.nx, &dummy);
    const int cy = diag_axis(py, a.g.oy, a.g.cs, a.g.ny, &dummy);
    const int cz = diag_axis(pz, a.g.oz, a.g.cs, a.g.nz, &dummy);
    const double wd = 21.0 / (16.0 * M_PI * h * h * h);
    double num = 0.0, den = 0.0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy) {
            const int czn = cz + dz, cyn = cy + dy;
            if (czn < 0 || czn >= a.g.nz || cyn < 0 || cyn >= a.g.ny) continue;
            const int64_t rb = lin_cell(0, cyn, czn, a.g.nx, a.g.ny);
            const int xl = cx > 0 ? cx - 1 : 0, xh = cx + 1 < a.g.nx ? cx + 1 : a.g.nx - 1;
            const uint32_t js = a.cell_start[rb + xl], je = a.cell_start[rb + xh + 1];
            for (uint32_t j = js + threadIdx.x; j < je; j += kDiagThreads) {
                if ((a.id[j] >> 31) != 0) continue;
                const double dx = a.x[j] - px, dy_ = a.y[j] - py, dz_ = a.z[j] - pz;
                const double r2 = (dx * dx + dy_ * dy_) + dz_ * dz_;
                if (!(r2 < a.r2max)) continue;
                const double w = wendland(sqrt(r2) / h, wd);
                const double rho = density_at(a, j);
                const double P = a.B * (pow(rho / a.rho0, a.gamma) - 1.0);
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

int launch_diag(const sph_params &p, const sph_state &s, const Ws &w, const double *probes,
                int32_t np, sph_diag *out, double *probe_p, hipStream_t st) {
    DiagArgs a;
    a.n = s.n;
    a.x = s.x;
    a.y = s.y;
    a.z = s.z;
    a.ux = s.ux;
    a.uy = s.uy;
    a.uz = s.uz;
    a.rho = s.rho;
    a.id = s.id;
    a.cell_start = w.cell_start();
    a.mixed = p.precision == SPH_MIXED;
    a.g = grid_of(p);
    a.mass = p.mass;
    a.rho0 = p.rho0;
    a.B = p.rho0 * p.c0 * p.c0 / p.gamma;
    a.gamma = p.gamma;
    a.gx = p.g[0];
    a.gy = p.g[1];
    a.gz = p.g[2];
    a.r2max = 4.0 * p.h * p.h;
    a.part = w.diag_part();
    double *res = w.diag_part() + (size_t)kDiagBlocks * kDiagFields;
    double *pts = res + kDiagFields;
    double *pout = pts + 3 * kMaxProbes;
    hipLaunchKernelGGL(k_diag_partial, dim3(kDiagBlocks), dim3(kDiagThreads), 0, st, a);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kDiagThreads), 0, st, a.part, kDiagBlocks, res);
    if (int rc = launch_check("diagnostics")) return rc;
    if (np > 0) {
        if (int rc = hip_check(hipMemcpyAsync(pts, probes, sizeof(double) * 3 * np,
                                              hipMemcpyHostToDevice, st),
                               "probe upload"))
            return rc;
        hipLaunchKernelGGL(k_probes, dim3(np), dim3(kDiagThreads), 0, st, a, pts, p.h, pout);
        if (int rc = launch_check("probes")) return rc;
    }
    double host[kDiagFields];
    DevScalars sc;
    if (int rc = hip_check(hipMemcpyAsync(host, res, sizeof(host), hipMemcpyDeviceToHost, st),
                           "diagnostics download"))
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
    std::memset(out, 0, sizeof(*out));
    out->mass = host[F_MASS];
    out->mom[0] = host[F_PX];
    out->mom[1] = host[F_PY];
    out->mom[2] = host[F_PZ];
    out->e_kin = host[F_EKIN];
    out->e_pot = host[F_EPOT];
    out->e_int = host[F_EINT];
    out->umax = host[F_UMAX];
    out->x_front = host[F_FRONT];
    out->dt_cfl = sc.dt_cfl;
    out->dt_last = sc.dt_last;
    out->time = sc.time;
    out->n = s.n;
    out->n_fluid = (int64_t)host[F_NFLUID];
    out->n_outside = (int64_t)host[F_OUTSIDE];
    out->n_nonfinite = (int64_t)host[F_NONFIN];
    out->steps = sc.steps;
    out->pairs_ff = (int64_t)sc.pairs[0];
    out->pairs_fb = (int64_t)sc.pairs[1];
    out->pairs_bf = (int64_t)sc.pairs[2];
    uint32_t flags = 0;
    if (out->n_nonfinite > 0) flags |= SPH_FLAG_NONFINITE;
    if (out->n_outside > 0) flags |= SPH_FLAG_OUTSIDE;
    if (host[F_DENS] > 0.1) flags |= SPH_FLAG_DENSITY;
    if (sc.dt_cfl_violation) flags |= SPH_FLAG_DT_CFL;
    out->flags = flags;
    return 0;
}

}  // namespace wcsph
