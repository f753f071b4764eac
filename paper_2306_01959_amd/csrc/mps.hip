// Explicit MPS operators (Section 2, MPS subsection) on the cell list: the
// weight w = r_e / r - 1 (eq. mpsw), the particle number density n_i = sum w
// (eq. mpspnd), the gradient (eq. mpsgrad) and Laplacian (eq. mpslap, with
// lambda0 of eq. mpslambda) of a scalar field, and the neighbourhood-centroid
// deviation sigma_i (eq. mpssigmai2) with the two-criteria free-surface test
// n_i < beta1 n0 and sigma_i > rho1 l0 (eqs. mpsni, mpsisgmai1).
//
// Neighbours of i are all other particles, fluid and wall, with
// 0 < |r_j - r_i| < r_e (coincident particles, where w is unbounded, are left
// out).  One thread per particle walks the fluid and the boundary halves of
// its 27-cell stencil (the cells must be at least r_e wide); FP64 throughout.
// The pressure Poisson solve of the method is not part of this library.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "common.h"

namespace wcsph {

struct MpsArgs {
    int64_t n;
    const double *x, *y, *z;
    const uint32_t *cell_start;
    Inst ip;
    double re, n0, lambda0, beta1, rho1l0;
    const double *phi;
    double *pnd, *lap, *gx, *gy, *gz, *sigma;
    int32_t *surface;
};

__device__ __forceinline__ int mps_cell(double v, double o, double cs, int n) {
    const double f = floor((v - o) / cs);
    if (!(f >= 0.0)) return 0;
    if (f > (double)(n - 1)) return n - 1;
    return (int)f;
}

__device__ __forceinline__ double mps_r2(double dx, double dy, double dz) {
#pragma clang fp contract(off)
    const double a = dx * dx;
    const double b = dy * dy;
    const double c = dz * dz;
    return (a + b) + c;
}

__global__ __launch_bounds__(256) void k_mps(MpsArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const Inst &ip = a.ip;
    const double xi = a.x[i], yi = a.y[i], zi = a.z[i];
    const int cx = mps_cell(xi, ip.ox, ip.cs, ip.nx);
    const int cy = mps_cell(yi, ip.oy, ip.cs, ip.ny);
    const int cz = mps_cell(zi, ip.oz, ip.cs, ip.nz);
    const double re = a.re, re2 = re * re;
    const bool field = a.phi != nullptr;
    const double phii = field ? a.phi[i] : 0.0;
    double sw = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    double sl = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    const int xl = cx > 0 ? cx - 1 : 0, xh = cx + 1 < ip.nx ? cx + 1 : ip.nx - 1;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy) {
            const int czn = cz + dz, cyn = cy + dy;
            if (czn < 0 || czn >= ip.nz || cyn < 0 || cyn >= ip.ny) continue;
            for (uint32_t half = 0; half < 2; ++half) {
                const uint32_t hb =
                    half_row_key(ip.cell_base, ip.nx, (uint32_t)(czn * ip.ny + cyn), half);
                const uint32_t js = a.cell_start[hb + xl], je = a.cell_start[hb + xh + 1];
                for (uint32_t j = js; j < je; ++j) {
                    if ((int64_t)j == i) continue;
                    const double rx = a.x[j] - xi, ry = a.y[j] - yi, rz = a.z[j] - zi;
                    const double r2 = mps_r2(rx, ry, rz);
                    if (!(r2 < re2) || !(r2 > 0.0)) continue;
                    const double w = re / sqrt(r2) - 1.0;
                    sw += w;
                    sx += rx * w;
                    sy += ry * w;
                    sz += rz * w;
                    if (field) {
                        const double d = a.phi[j] - phii;
                        sl += d * w;
                        gx += d * rx * w / r2;
                        gy += d * ry * w / r2;
                        gz += d * rz * w / r2;
                    }
                }
            }
        }
    const double sig = sw > 0.0 ? sqrt(mps_r2(sx, sy, sz)) / sw : 0.0;
    if (a.pnd) a.pnd[i] = sw;
    if (a.sigma) a.sigma[i] = sig;
    if (a.surface) a.surface[i] = (sw < a.beta1 * a.n0 && sig > a.rho1l0) ? 1 : 0;
    if (field && a.lap) a.lap[i] = 6.0 / (a.lambda0 * a.n0) * sl;
    if (field && a.gx) {
        a.gx[i] = 3.0 / a.n0 * gx;
        a.gy[i] = 3.0 / a.n0 * gy;
        a.gz[i] = 3.0 / a.n0 * gz;
    }
}

int launch_mps(const Problem &P, const sph_state &s, const Ws &w, const sph_mps *m,
               const double *phi, double *pnd, double *lap, double *grad, double *sigma,
               int32_t *surface, hipStream_t st) {
    MpsArgs a;
    a.n = s.n;
    a.x = s.x;
    a.y = s.y;
    a.z = s.z;
    a.cell_start = w.cell_start();
    a.ip = P.host[0];
    a.re = m->re;
    a.n0 = m->n0;
    a.lambda0 = m->lambda0;
    a.beta1 = m->beta1;
    a.rho1l0 = m->rho1 * m->l0;
    a.phi = phi;
    a.pnd = pnd;
    a.lap = lap;
    a.gx = grad;
    a.gy = grad ? grad + s.n : nullptr;
    a.gz = grad ? grad + 2 * s.n : nullptr;
    a.sigma = sigma;
    a.surface = surface;
    hipLaunchKernelGGL(k_mps, dim3((unsigned)((s.n + 255) / 256)), dim3(256), 0, st, a);
    return launch_check("mps operators");
}

// n0 and lambda0 of the fully filled support on the cubic lattice of
// spacing l0 (eqs. mpspnd, mpslambda): sums over the lattice points within
// r_e of the origin, on the host.
void mps_lattice_constants(double l0, double re, double *n0, double *lambda0) {
    const int kmax = (int)std::ceil(re / l0) + 1;
    double sw = 0.0, sr2w = 0.0;
    for (int a = -kmax; a <= kmax; ++a)
        for (int b = -kmax; b <= kmax; ++b)
            for (int c = -kmax; c <= kmax; ++c) {
                const double dx = a * l0, dy = b * l0, dz = c * l0;
                const double aa = dx * dx, bb = dy * dy, cc = dz * dz;
                const double r2 = (aa + bb) + cc;
                const double r = std::sqrt(r2);
                if (!(r > 0.0) || !(r < re)) continue;
                const double wgt = re / r - 1.0;
                sw += wgt;
                sr2w += r2 * wgt;
            }
    *n0 = sw;
    *lambda0 = sr2w / sw;
}

}  // namespace wcsph
