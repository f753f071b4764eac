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
// A wave's particles are consecutive in cell order, so they usually share a
// cell row and their stencil rows overlap: the wave then stages each stencil
// row's candidates {x, y, z, phi} once in LDS (one coalesced load per
// candidate instead of four gathers per lane) and every lane reads its own
// window of them; a wave that spans two rows, or a row range too long for the
// staging buffer, loads from memory as before.  Each lane visits the same
// candidates in the same order either way, so the sums are identical.
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

constexpr int kMpsThreads = 256;
constexpr int kMpsStage = 256;  // candidates a wave stages per stencil row

__global__ __launch_bounds__(kMpsThreads) void k_mps(MpsArgs a) {
    __shared__ double4 stage[kMpsThreads / kWave][kMpsStage];
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // lanes past the end take part in the staging only (n >= 1); lane 0 is
    // active in every wave that has an active lane
    const bool act = i < a.n;
    if (__ballot(act) == 0ull) return;  // the whole wave: no barrier follows
    const int64_t ti = act ? i : a.n - 1;
    const Inst &ip = a.ip;
    const double xi = a.x[ti], yi = a.y[ti], zi = a.z[ti];
    const int cx = mps_cell(xi, ip.ox, ip.cs, ip.nx);
    const int cy = mps_cell(yi, ip.oy, ip.cs, ip.ny);
    const int cz = mps_cell(zi, ip.oz, ip.cs, ip.nz);
    const double re = a.re, re2 = re * re;
    const bool field = a.phi != nullptr;
    const double phii = field ? a.phi[ti] : 0.0;
    // one cell row for the whole wave (its active lanes)?
    const int row = cz * ip.ny + cy;
    const int row0 = __builtin_amdgcn_readfirstlane(row);
    const bool one_row = __ballot(act && row != row0) == 0ull;
    int cxlo = act ? cx : ip.nx, cxhi = act ? cx : -1;
    for (int off = 1; off < kWave; off <<= 1) {
        const int lo = __shfl_xor(cxlo, off, kWave), hi = __shfl_xor(cxhi, off, kWave);
        cxlo = lo < cxlo ? lo : cxlo;
        cxhi = hi > cxhi ? hi : cxhi;
    }
    const int ulo = cxlo > 0 ? cxlo - 1 : 0, uhi = cxhi + 1 < ip.nx ? cxhi + 1 : ip.nx - 1;
    // the stencil's centre row: lane 0's for the whole wave when they share it
    // (then the lanes past the end follow it too)
    const int cz0 = one_row ? __builtin_amdgcn_readfirstlane(cz) : cz;
    const int cy0 = one_row ? __builtin_amdgcn_readfirstlane(cy) : cy;
    double sw = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    double sl = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    // (the particle itself is at r = 0 and is left out with the coincident ones)
    auto visit = [&](double xj, double yj, double zj, double phj) {
        const double rx = xj - xi, ry = yj - yi, rz = zj - zi;
        const double r2 = mps_r2(rx, ry, rz);
        if (!(r2 < re2) || !(r2 > 0.0)) return;
        // one square root and one division per pair: w = r_e / r - 1 and
        // 1 / r^2 from 1 / r (a few ulp from the textbook order)
        const double ir = 1.0 / sqrt(r2);
        const double w = re * ir - 1.0;
        sw += w;
        sx += rx * w;
        sy += ry * w;
        sz += rz * w;
        if (field) {
            const double d = phj - phii;
            sl += d * w;
            const double f = d * w * (ir * ir);
            gx += f * rx;
            gy += f * ry;
            gz += f * rz;
        }
    };
    const int xl = cx > 0 ? cx - 1 : 0, xh = cx + 1 < ip.nx ? cx + 1 : ip.nx - 1;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy) {
            const int czn = cz0 + dz, cyn = cy0 + dy;
            const bool in_grid = czn >= 0 && czn < ip.nz && cyn >= 0 && cyn < ip.ny;
            for (uint32_t half = 0; half < 2; ++half) {
                const uint32_t hb =
                    in_grid ? half_row_key(ip, (uint32_t)(czn * ip.ny + cyn), half) : 0u;
                uint32_t js = 0, je = 0;
                if (in_grid && act) {
                    js = a.cell_start[hb + xl];
                    je = a.cell_start[hb + xh + 1];
                }
                if (one_row) {
                    // wave-uniform: the same stencil row for every lane
                    if (!in_grid) continue;
                    const uint32_t u0 = a.cell_start[hb + ulo], u1 = a.cell_start[hb + uhi + 1];
                    if (u1 - u0 <= (uint32_t)kMpsStage) {
                        for (uint32_t k = lane; k < u1 - u0; k += kWave) {
                            const uint32_t j = u0 + k;
                            stage[wv][k] = make_double4(a.x[j], a.y[j], a.z[j],
                                                       field ? a.phi[j] : 0.0);
                        }
                        wave_sync();
                        for (uint32_t j = js; j < je; ++j) {
                            const double4 c = stage[wv][j - u0];
                            visit(c.x, c.y, c.z, c.w);
                        }
                        wave_sync();  // the next row overwrites the buffer
                        continue;
                    }
                }
                for (uint32_t j = js; j < je; ++j)
                    visit(a.x[j], a.y[j], a.z[j], field ? a.phi[j] : 0.0);
            }
        }
    if (!act) return;
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
    hipLaunchKernelGGL(k_mps, dim3((unsigned)((s.n + kMpsThreads - 1) / kMpsThreads)),
                       dim3(kMpsThreads), 0, st, a);
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
