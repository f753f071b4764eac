// Cell-linked list on the GPU: hash -> stable radix sort -> reorder + view.
//
// The neighbour set of the method is every j with |r_j - r_i| < 2h
// (Wendland support, Section 2.2).  Particles are binned into cells of edge
// cs >= 2h, so every neighbour lies in the 27 cells around a particle's own.
// Cells are numbered x-fastest, which makes the three cells of a stencil row
// contiguous in sorted order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "common.h"

namespace wcsph {

// ---------------------------------------------------------------- encode

__device__ __forceinline__ int axis_cell(double v, double o, double cs, int n) {
    // floor((v - o) / cs) with an IEEE division, clamped to [0, n - 1]
    // (NaN -> 0).  Clamping is monotone, so pairs closer than cs still land
    // in adjacent cells.
    double f = floor((v - o) / cs);
    if (!(f >= 0.0)) return 0;
    if (f > (double)(n - 1)) return n - 1;
    return (int)f;
}

__global__ void k_encode(const double *__restrict__ x, const double *__restrict__ y,
                         const double *__restrict__ z, int64_t n, Grid g,
                         uint32_t *__restrict__ keys) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int cx = axis_cell(x[i], g.ox, g.cs, g.nx);
    int cy = axis_cell(y[i], g.oy, g.cs, g.ny);
    int cz = axis_cell(z[i], g.oz, g.cs, g.nz);
    keys[i] = (uint32_t)lin_cell(cx, cy, cz, g.nx, g.ny);
}

int launch_encode(const sph_params &p, const sph_state &s, const Ws &w, hipStream_t st) {
    int64_t n = s.n;
    int blocks = (int)((n + 255) / 256);
    hipLaunchKernelGGL(k_encode, dim3(blocks), dim3(256), 0, st, s.x, s.y, s.z, n, grid_of(p),
                       w.keys());
    return launch_check("encode");
}

// ------------------------------------------------------------ radix sort
//
// LSD radix sort of (32-bit key, 32-bit index) pairs, 8-bit digits.  Per
// pass: tile histograms -> one exclusive scan over (digit, tile) -> stable
// scatter.  Ranks inside a tile come from wave-wide digit matching (eight
// ballots), so a tile's keys keep their input order: the sort is stable and
// deterministic.

__device__ __forceinline__ uint64_t lanemask_lt() {
    uint32_t lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Lanes of the wave whose digit equals this lane's (restricted to `valid`).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t valid) {
    uint64_t peers = valid;
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        uint64_t bal = __ballot((d >> b) & 1u);
        peers &= ((d >> b) & 1u) ? bal : ~bal;
    }
    return peers;
}

__global__ __launch_bounds__(kSortThreads) void k_sort_hist(const uint32_t *__restrict__ keys,
                                                            int64_t n, int shift,
                                                            uint32_t *__restrict__ hist,
                                                            int ntiles) {
    __shared__ uint32_t h[kRadix];
    const int tid = threadIdx.x;
    for (int d = tid; d < kRadix; d += kSortThreads) h[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int it = 0; it < kSortItems; ++it) {
        int64_t idx = base + (int64_t)it * kSortThreads + tid;
        bool ok = idx < n;
        uint32_t d = ok ? (keys[idx] >> shift) & (kRadix - 1) : 0u;
        uint64_t peers = match_digit(d, __ballot(ok));
        if (ok && (peers & lanemask_lt()) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    for (int d = tid; d < kRadix; d += kSortThreads) hist[(int64_t)d * ntiles + blockIdx.x] = h[d];
}

// Exclusive scan of m values in place, one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan_excl(uint32_t *__restrict__ a, int64_t m) {
    __shared__ uint32_t sums[1024];
    const int t = threadIdx.x;
    const int64_t per = (m + 1023) / 1024;
    const int64_t b = t * per;
    const int64_t e = b + per < m ? b + per : m;
    uint32_t s = 0;
    for (int64_t k = b; k < e; ++k) s += a[k];
    sums[t] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the 1024 partial sums
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t v = t >= off ? sums[t - off] : 0u;
        __syncthreads();
        sums[t] += v;
        __syncthreads();
    }
    uint32_t run = t > 0 ? sums[t - 1] : 0u;
    for (int64_t k = b; k < e; ++k) {
        uint32_t v = a[k];
        a[k] = run;
        run += v;
    }
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout,
    uint32_t *__restrict__ vout, int64_t n, int shift, const uint32_t *__restrict__ hist,
    int ntiles) {
    constexpr int kWaves = kSortThreads / kWave;
    __shared__ uint32_t run[kRadix];          // next free slot per digit for this tile
    __shared__ uint32_t wpos[kWaves][kRadix]; // per-wave counts, then start slots
    const int tid = threadIdx.x;
    const int w = tid / kWave;
    for (int d = tid; d < kRadix; d += kSortThreads) {
        run[d] = hist[(int64_t)d * ntiles + blockIdx.x];
        for (int k = 0; k < kWaves; ++k) wpos[k][d] = 0;
    }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const uint64_t lt = lanemask_lt();
    for (int it = 0; it < kSortItems; ++it) {
        int64_t idx = base + (int64_t)it * kSortThreads + tid;
        bool ok = idx < n;
        uint32_t key = ok ? kin[idx] : 0u;
        uint32_t val = ok ? (vin ? vin[idx] : (uint32_t)idx) : 0u;
        uint32_t d = (key >> shift) & (kRadix - 1);
        uint64_t peers = match_digit(d, __ballot(ok));
        uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (ok && rank == 0) wpos[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        for (int dd = tid; dd < kRadix; dd += kSortThreads) {
            uint32_t r = run[dd];
            for (int k = 0; k < kWaves; ++k) {
                uint32_t c = wpos[k][dd];
                wpos[k][dd] = r;
                r += c;
            }
            run[dd] = r;
        }
        __syncthreads();
        if (ok) {
            uint32_t pos = wpos[w][d] + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        for (int dd = tid; dd < kRadix; dd += kSortThreads)
            for (int k = 0; k < kWaves; ++k) wpos[k][dd] = 0;
        __syncthreads();
    }
}

int launch_sort(const Ws &w, hipStream_t st, uint32_t **sorted_keys, uint32_t **perm) {
    const int64_t n = w.L.n;
    const int ntiles = (int)w.L.ntiles;
    const int passes = w.L.key_bits <= 0 ? 1 : (w.L.key_bits + kRadixBits - 1) / kRadixBits;
    uint32_t *kin = w.keys(), *kout = w.keys_alt();
    uint32_t *vbuf[2] = {w.vals(), w.vals_alt()};
    uint32_t *vin = nullptr;  // first pass ranks the identity permutation
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = pass * kRadixBits;
        uint32_t *vout = vbuf[pass & 1];
        hipLaunchKernelGGL(k_sort_hist, dim3(ntiles), dim3(kSortThreads), 0, st, kin, n, shift,
                           w.hist(), ntiles);
        hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, st, w.hist(),
                           (int64_t)kRadix * ntiles);
        hipLaunchKernelGGL(k_sort_scatter, dim3(ntiles), dim3(kSortThreads), 0, st, kin, vin,
                           kout, vout, n, shift, w.hist(), ntiles);
        if (int rc = launch_check("radix sort")) return rc;
        uint32_t *t = kin;
        kin = kout;
        kout = t;
        vin = vout;
    }
    *sorted_keys = kin;
    *perm = vin;
    return 0;
}

// ----------------------------------------------------- reorder and view

struct ReorderArgs {
    const uint32_t *perm;
    const uint32_t *keys;
    int64_t n;
    // source arrays
    const double *x, *y, *z, *ux, *uy, *uz, *uxm, *uym, *uzm;
    const void *rho, *rhom;
    const uint32_t *id;
    // destination arrays
    double *x2, *y2, *z2, *ux2, *uy2, *uz2, *uxm2, *uym2, *uzm2;
    void *rho2, *rhom2;
    uint32_t *id2;
    // view
    void *v0, *v1, *v2;
    Grid g;
    double rho0, B, gamma, c0;
    int c_const;
};

// Offset of coordinate v from the centre of cell c, computed in FP64 with
// one rounding per operation (no contraction) and rounded once to FP32.
__device__ __forceinline__ float cell_offset(double v, double o, int c, double cs) {
#pragma clang fp contract(off)
    double t = v - o;
    double ctr = ((double)c + 0.5) * cs;
    return (float)(t - ctr);
}

template <bool kMixed>
__global__ void k_reorder(ReorderArgs a) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const uint32_t src = a.perm[k];
    const double x = a.x[src], y = a.y[src], z = a.z[src];
    const double ux = a.ux[src], uy = a.uy[src], uz = a.uz[src];
    const uint32_t id = a.id[src];
    a.x2[k] = x;
    a.y2[k] = y;
    a.z2[k] = z;
    a.ux2[k] = ux;
    a.uy2[k] = uy;
    a.uz2[k] = uz;
    a.uxm2[k] = a.uxm[src];
    a.uym2[k] = a.uym[src];
    a.uzm2[k] = a.uzm[src];
    a.id2[k] = id;
    const bool bnd = (id >> 31) != 0;
    if constexpr (kMixed) {
        const float dr = static_cast<const float *>(a.rho)[src];
        static_cast<float *>(a.rho2)[k] = dr;
        static_cast<float *>(a.rhom2)[k] = static_cast<const float *>(a.rhom)[src];
        const uint32_t c = a.keys[k];
        const int cx = (int)(c % (uint32_t)a.g.nx);
        const int cy = (int)((c / (uint32_t)a.g.nx) % (uint32_t)a.g.ny);
        const int cz = (int)(c / ((uint32_t)a.g.nx * (uint32_t)a.g.ny));
        const double xr = (double)dr / a.rho0;
        const double l1p = log1p(xr);
        const double P = a.B * expm1(a.gamma * l1p);
        const double cs = a.c_const ? a.c0 : a.c0 * exp(0.5 * (a.gamma - 1.0) * l1p);
        const double inv = 1.0 / (a.rho0 + (double)dr);
        float4 v0 = make_float4(cell_offset(x, a.g.ox, cx, a.g.cs), cell_offset(y, a.g.oy, cy, a.g.cs),
                                cell_offset(z, a.g.oz, cz, a.g.cs), dr);
        float4 v1 = make_float4((float)ux, (float)uy, (float)uz, (float)P);
        float2 v2 = make_float2((float)inv, bnd ? -(float)cs : (float)cs);
        static_cast<float4 *>(a.v0)[k] = v0;
        static_cast<float4 *>(a.v1)[k] = v1;
        static_cast<float2 *>(a.v2)[k] = v2;
    } else {
        const double rho = static_cast<const double *>(a.rho)[src];
        static_cast<double *>(a.rho2)[k] = rho;
        static_cast<double *>(a.rhom2)[k] = static_cast<const double *>(a.rhom)[src];
        const double r = rho / a.rho0;
        const double P = a.B * (pow(r, a.gamma) - 1.0);
        const double cs = a.c_const ? a.c0 : a.c0 * pow(r, 0.5 * (a.gamma - 1.0));
        double4 v0 = make_double4(x, y, z, rho);
        double4 v1 = make_double4(ux, uy, uz, P);
        double2 v2 = make_double2(1.0 / rho, bnd ? -cs : cs);
        static_cast<double4 *>(a.v0)[k] = v0;
        static_cast<double4 *>(a.v1)[k] = v1;
        static_cast<double2 *>(a.v2)[k] = v2;
    }
}

int launch_reorder(const sph_params &p, sph_state &s, const Ws &w, const uint32_t *keys,
                   const uint32_t *perm, hipStream_t st) {
    ReorderArgs a;
    a.perm = perm;
    a.keys = keys;
    a.n = s.n;
    a.x = s.x; a.y = s.y; a.z = s.z;
    a.ux = s.ux; a.uy = s.uy; a.uz = s.uz;
    a.uxm = s.uxm; a.uym = s.uym; a.uzm = s.uzm;
    a.rho = s.rho; a.rhom = s.rhom; a.id = s.id;
    a.x2 = s.x_alt; a.y2 = s.y_alt; a.z2 = s.z_alt;
    a.ux2 = s.ux_alt; a.uy2 = s.uy_alt; a.uz2 = s.uz_alt;
    a.uxm2 = s.uxm_alt; a.uym2 = s.uym_alt; a.uzm2 = s.uzm_alt;
    a.rho2 = s.rho_alt; a.rhom2 = s.rhom_alt; a.id2 = s.id_alt;
    a.v0 = w.base + w.L.view0;
    a.v1 = w.base + w.L.view1;
    a.v2 = w.base + w.L.view2;
    a.g = grid_of(p);
    a.rho0 = p.rho0;
    a.B = p.rho0 * p.c0 * p.c0 / p.gamma;
    a.gamma = p.gamma;
    a.c0 = p.c0;
    a.c_const = p.c_mode == SPH_C_CONST;
    int blocks = (int)((s.n + 255) / 256);
    if (p.precision == SPH_MIXED)
        hipLaunchKernelGGL(k_reorder<true>, dim3(blocks), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_reorder<false>, dim3(blocks), dim3(256), 0, st, a);
    if (int rc = launch_check("reorder")) return rc;
    // the gathered arrays are now current
    auto swp = [](auto &u, auto &v) { auto t = u; u = v; v = t; };
    swp(s.x, s.x_alt); swp(s.y, s.y_alt); swp(s.z, s.z_alt);
    swp(s.ux, s.ux_alt); swp(s.uy, s.uy_alt); swp(s.uz, s.uz_alt);
    swp(s.uxm, s.uxm_alt); swp(s.uym, s.uym_alt); swp(s.uzm, s.uzm_alt);
    swp(s.rho, s.rho_alt); swp(s.rhom, s.rhom_alt); swp(s.id, s.id_alt);
    return 0;
}

// ------------------------------------------------------------ cell table

// cell_start[c] = first sorted position whose key >= c, for c in [0, ncells]
// (lower bound by binary search; empty cells get the start of the next one).
__global__ void k_cell_table(const uint32_t *__restrict__ keys, int64_t n, int64_t ncells,
                             uint32_t *__restrict__ start) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c > ncells) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((int64_t)keys[mid] < c)
            lo = mid + 1;
        else
            hi = mid;
    }
    start[c] = (uint32_t)lo;
}

int launch_cell_table(const sph_params &p, const Ws &w, const uint32_t *keys, hipStream_t st) {
    (void)p;
    int64_t m = w.L.ncells + 1;
    int blocks = (int)((m + 255) / 256);
    hipLaunchKernelGGL(k_cell_table, dim3(blocks), dim3(256), 0, st, keys, w.L.n, w.L.ncells,
                       w.cell_start());
    return launch_check("cell table");
}

// ------------------------------------------------------------ chunk list
//
// The interaction works on chunks: up to 64 consecutive sorted particles of
// one cell row (fixed cy, cz).  One workgroup scans the rows, writes every
// chunk {start, end, row, 0} and the chunk count, and resets the running
// minimum of the time-step bound and the chunk counter for the interaction
// that follows.
__global__ __launch_bounds__(1024) void k_chunks(const uint32_t *__restrict__ start, int nx,
                                                 int64_t nrows, int4 *__restrict__ chunks,
                                                 DevScalars *sc) {
    __shared__ uint32_t sums[1024];
    __shared__ uint32_t carry;
    const int t = threadIdx.x;
    if (t == 0) {
        carry = 0;
        sc->dt_min_bits = 0x7ff0000000000000ull;  // +inf
        sc->work = 0;
    }
    __syncthreads();
    for (int64_t r0 = 0; r0 < nrows; r0 += 1024) {
        int64_t r = r0 + t;
        uint32_t b = 0, e = 0, nch = 0;
        if (r < nrows) {
            b = start[r * nx];
            e = start[(r + 1) * nx];
            nch = (e - b + kChunk - 1) / kChunk;
        }
        sums[t] = nch;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            uint32_t v = t >= off ? sums[t - off] : 0u;
            __syncthreads();
            sums[t] += v;
            __syncthreads();
        }
        uint32_t first = carry + sums[t] - nch;
        for (uint32_t k = 0; k < nch; ++k) {
            uint32_t s0 = b + k * kChunk;
            uint32_t s1 = s0 + kChunk < e ? s0 + kChunk : e;
            chunks[first + k] = make_int4((int)s0, (int)s1, (int)r, 0);
        }
        __syncthreads();
        if (t == 1023) carry += sums[1023];
        __syncthreads();
    }
    if (t == 0) sc->nchunks = carry;
}

int launch_chunks(const sph_params &p, const Ws &w, hipStream_t st) {
    hipLaunchKernelGGL(k_chunks, dim3(1), dim3(1024), 0, st, w.cell_start(), p.dims[0],
                       w.L.nrows, w.chunks(), w.scalars());
    return launch_check("chunk list");
}

}  // namespace wcsph
