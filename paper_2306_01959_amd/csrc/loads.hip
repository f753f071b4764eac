// Loads on solids (Section 3): the force on a set of wall particles and the
// pressure impulse at probe points.
//
// Force.  The paper obtains the force on the block as the sum, over the wall
// particles of its weather side, of each particle's acceleration from the
// momentum equation (eq. sphu) times its mass; the wall particles do not move
// with it.  Here the set is every boundary particle inside an axis-aligned
// box, and a particle's acceleration is the pressure and viscosity terms of
// eq. sphu (eq. pi, cpmu, tait) over its fluid neighbours, in FP64 from the
// state arrays, without the body force.  One block per cell row that meets
// the box walks the row's boundary particles inside the box and the fluid
// halves of their 27-cell stencils; per-block sums in a fixed order, then
// one block adds the blocks in order, so the result is bit-reproducible.
//
// Impulse.  I_p = integral of P dt at each probe (Table 2's quantity),
// accumulated on the device by the trapezoidal rule over the samples taken
// by successive calls, with the simulated time the steps accumulated.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "common.h"

namespace wcsph {

constexpr int kLoadThreads = 256;

struct ForceArgs {
    const double *x, *y, *z, *ux, *uy, *uz;
    const void *rho;
    const uint32_t *id;
    const uint32_t *cell_start;
    int mixed;
    Inst ip;
    double bx0, bx1, by0, by1, bz0, bz1;  // the box
    int cx0, cx1, cy0, cz0, nby;          // its cells
    double *part;                         // 4 doubles per block
};

__device__ __forceinline__ double load_density(const ForceArgs &a, int64_t i) {
    return a.mixed ? a.ip.rho0 + (double)static_cast<const float *>(a.rho)[i]
                   : static_cast<const double *>(a.rho)[i];
}

// eq. tait; with the paper's gamma = 7 the powers are products (a few ulp
// from pow, at a fraction of its cost: the pair loop evaluates them per pair)
__device__ __forceinline__ double load_pressure(const Inst &ip, double rho) {
    const double x = rho / ip.rho0;
    if (ip.gamma == 7.0) {
        const double x2 = x * x, x4 = x2 * x2;
        return ip.B * (x4 * x2 * x - 1.0);
    }
    return ip.B * (pow(x, ip.gamma) - 1.0);
}

__device__ __forceinline__ double load_sound(const Inst &ip, double rho) {
    if (ip.c_const) return ip.c0;
    const double x = rho / ip.rho0;
    if (ip.gamma == 7.0) return ip.c0 * (x * x * x);
    return ip.c0 * pow(x, 0.5 * (ip.gamma - 1.0));
}

// The neighbour predicate's r^2 = (dx dx + dy dy) + dz dz without contraction.
__device__ __forceinline__ double load_r2(double dx, double dy, double dz) {
#pragma clang fp contract(off)
    const double a = dx * dx;
    const double b = dy * dy;
    const double c = dz * dz;
    return (a + b) + c;
}

__global__ __launch_bounds__(kLoadThreads) void k_boundary_force(ForceArgs a) {
    __shared__ double red[4][kLoadThreads / kWave];
    const Inst &ip = a.ip;
    const int cy = a.cy0 + (int)blockIdx.x % a.nby;
    const int cz = a.cz0 + (int)blockIdx.x / a.nby;
    // this row's boundary particles in the box's cells
    const uint32_t hb = half_row_key(ip, (uint32_t)(cz * ip.ny + cy), 1);
    const uint32_t i0 = a.cell_start[hb + a.cx0], i1 = a.cell_start[hb + a.cx1 + 1];
    const double h = ip.h, m = ip.mass, eta2 = ip.eta2;
    const double inv_h = 1.0 / h, fk = 5.0 * ip.wd / (h * h);
    double fx = 0.0, fy = 0.0, fz = 0.0, cnt = 0.0;
    for (uint32_t i = i0 + threadIdx.x; i < i1; i += kLoadThreads) {
        const double xi = a.x[i], yi = a.y[i], zi = a.z[i];
        if (!(xi >= a.bx0 && xi <= a.bx1 && yi >= a.by0 && yi <= a.by1 && zi >= a.bz0 &&
              zi <= a.bz1))
            continue;
        cnt += 1.0;
        const double rhoi = load_density(a, i);
        const double Pi = load_pressure(ip, rhoi), Ci = load_sound(ip, rhoi);
        const double uxi = a.ux[i], uyi = a.uy[i], uzi = a.uz[i];
        // the particle's cell along x, clamped to the grid as the sort's
        // (its row gives the cell along y and z)
        double ax = 0.0, ay = 0.0, az = 0.0;
        const double fcx = floor((xi - ip.ox) / ip.cs);
        const int pcx = !(fcx >= 0.0) ? 0 : (fcx > (double)(ip.nx - 1) ? ip.nx - 1 : (int)fcx);
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy) {
                const int czn = cz + dz, cyn = cy + dy;
                if (czn < 0 || czn >= ip.nz || cyn < 0 || cyn >= ip.ny) continue;
                const uint32_t fb = half_row_key(ip, (uint32_t)(czn * ip.ny + cyn), 0);
                const int xl = pcx > 0 ? pcx - 1 : 0, xh = pcx + 1 < ip.nx ? pcx + 1 : ip.nx - 1;
                const uint32_t js = a.cell_start[fb + xl], je = a.cell_start[fb + xh + 1];
                for (uint32_t j = js; j < je; ++j) {
                    const double rx = a.x[j] - xi, ry = a.y[j] - yi, rz = a.z[j] - zi;
                    const double r2 = load_r2(rx, ry, rz);
                    if (!(r2 < ip.r2max)) continue;
                    const double q = sqrt(r2) * inv_h;
                    const double t = 1.0 - 0.5 * q;
                    const double F = fk * (t * t * t);
                    const double vx = a.ux[j] - uxi, vy = a.uy[j] - uyi, vz = a.uz[j] - uzi;
                    const double vr = (vx * rx + vy * ry) + vz * rz;
                    const double rhoj = load_density(a, j);
                    double visc = 0.0;
                    if (vr < 0.0) {
                        const double mu = h * vr / (r2 + eta2);
                        visc = -ip.alpha * 0.5 * (Ci + load_sound(ip, rhoj)) * mu /
                               (0.5 * (rhoi + rhoj));
                    }
                    const double coef = m * ((Pi + load_pressure(ip, rhoj)) / (rhoi * rhoj) + visc);
                    ax -= coef * F * rx;
                    ay -= coef * F * ry;
                    az -= coef * F * rz;
                }
            }
        fx += m * ax;
        fy += m * ay;
        fz += m * az;
    }
    // fixed reduction: shuffles in each wave, then the waves in order
    double v[4] = {fx, fy, fz, cnt};
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    for (int f = 0; f < 4; ++f) {
        double s = v[f];
        for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
        if (lane == 0) red[f][w] = s;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double s = red[threadIdx.x][0];
        for (int q = 1; q < kLoadThreads / kWave; ++q) s += red[threadIdx.x][q];
        a.part[4 * (size_t)blockIdx.x + threadIdx.x] = s;
    }
}

// One block: the nb block sums in a fixed order -> out[0..3].
__global__ __launch_bounds__(kLoadThreads) void k_force_final(const double *__restrict__ part,
                                                              int nb, double *__restrict__ out) {
    __shared__ double red[4][kLoadThreads / kWave];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    for (int f = 0; f < 4; ++f) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += kLoadThreads) s += part[4 * (size_t)b + f];
        for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
        if (lane == 0) red[f][w] = s;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double s = red[threadIdx.x][0];
        for (int q = 1; q < kLoadThreads / kWave; ++q) s += red[threadIdx.x][q];
        out[threadIdx.x] = s;
    }
}

static int clamp_cell(double v, double o, double cs, int n) {
    const double f = std::floor((v - o) / cs);
    if (!(f >= 0.0)) return 0;
    if (f > (double)(n - 1)) return n - 1;
    return (int)f;
}

int launch_boundary_force(const Problem &P, const sph_state &s, const Ws &w, const double *box,
                          double *force, int64_t *count, hipStream_t st) {
    ForceArgs a;
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
    a.ip = P.host[0];
    const Inst &ip = a.ip;
    a.bx0 = box[0];
    a.bx1 = box[1];
    a.by0 = box[2];
    a.by1 = box[3];
    a.bz0 = box[4];
    a.bz1 = box[5];
    a.cx0 = clamp_cell(box[0], ip.ox, ip.cs, ip.nx);
    a.cx1 = clamp_cell(box[1], ip.ox, ip.cs, ip.nx);
    a.cy0 = clamp_cell(box[2], ip.oy, ip.cs, ip.ny);
    const int cy1 = clamp_cell(box[3], ip.oy, ip.cs, ip.ny);
    a.cz0 = clamp_cell(box[4], ip.oz, ip.cs, ip.nz);
    const int cz1 = clamp_cell(box[5], ip.oz, ip.cs, ip.nz);
    a.nby = cy1 - a.cy0 + 1;
    const int nb = a.nby * (cz1 - a.cz0 + 1);  // <= rows of the grid: fits the region
    a.part = w.loads();
    double *res = a.part + 4 * (size_t)w.L.nrows;
    hipLaunchKernelGGL(k_boundary_force, dim3(nb), dim3(kLoadThreads), 0, st, a);
    hipLaunchKernelGGL(k_force_final, dim3(1), dim3(kLoadThreads), 0, st, a.part, nb, res);
    if (int rc = launch_check("boundary force")) return rc;
    double host[4];
    if (int rc = hip_check(hipMemcpyAsync(host, res, sizeof(host), hipMemcpyDeviceToHost, st),
                           "force download"))
        return rc;
    if (int rc = hip_check(hipStreamSynchronize(st), "force sync")) return rc;
    force[0] = host[0];
    force[1] = host[1];
    force[2] = host[2];
    if (count) *count = (int64_t)host[3];
    return SPH_OK;
}

// I += (P_prev + P) / 2 (t - t_prev) for every probe, unless this is the
// first sample since init or reset, or the number of probes changed; then
// the integrals restart at zero.  Then P_prev = P, t_prev = t.
__global__ __launch_bounds__(kLoadThreads) void k_impulse(ImpulseState *imp, double *sum,
                                                          double *prev, const double *p, int np,
                                                          int reset, const InstState *ist) {
    const double t = ist[0].time;
    const bool acc = !reset && imp->has_prev && imp->np == np;
    const double dt = t - imp->t_prev;
    for (int a = threadIdx.x; a < np; a += kLoadThreads) {
        if (!acc) sum[a] = 0.0;
        else sum[a] += 0.5 * (prev[a] + p[a]) * dt;
        prev[a] = p[a];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        imp->t_prev = t;
        imp->has_prev = 1;
        imp->np = np;
    }
}

int launch_probe_impulse(const Problem &P, const sph_state &s, const Ws &w, const double *probes,
                         int32_t np, int32_t reset, double *probe_p, double *impulse,
                         hipStream_t st) {
    // the probe pressures go to the diagnostics' probe output slot
    double *pout = w.diag_part() + (size_t)P.host.size() * diag_blocks((int)P.host.size()) *
                                       kDiagFields +
                   (size_t)P.host.size() * kDiagFields + 3 * (size_t)kMaxProbes;
    if (int rc = launch_probes(P, s, w, probes, np, pout, st)) return rc;
    hipLaunchKernelGGL(k_impulse, dim3(1), dim3(kLoadThreads), 0, st, w.impulse(),
                       w.impulse_sum(), w.impulse_prev(), pout, np, reset, w.inst_state());
    if (int rc = launch_check("impulse")) return rc;
    if (int rc = hip_check(hipMemcpyAsync(probe_p, pout, sizeof(double) * np,
                                          hipMemcpyDeviceToHost, st),
                           "probe download"))
        return rc;
    if (int rc = hip_check(hipMemcpyAsync(impulse, w.impulse_sum(), sizeof(double) * np,
                                          hipMemcpyDeviceToHost, st),
                           "impulse download"))
        return rc;
    return hip_check(hipStreamSynchronize(st), "impulse sync");
}

}  // namespace wcsph
