// Pairwise WCSPH interaction (Section 2.2, eqs. sphu, pi, cpmu, sphw,
// sphrho, tait) and the per-particle time-step bound (eq. sphdt).
//
// Work decomposition: a chunk is up to 64 consecutive sorted particles of one
// cell row (fixed cy, cz; cells numbered x-fastest).  One wavefront owns a
// chunk, one target particle per lane.  The candidates of the chunk are the
// nine stencil rows (cy+dy, cz+dz) over cells [cx_first - 1, cx_last + 1],
// each a contiguous range of the sorted arrays.  The wave reads 64 candidates
// at a time (coalesced), drops those farther than 2h from the chunk's bounding
// box (a conservative cull) or irrelevant to its targets, compacts the rest
// into LDS with a ballot + popcount, and then every lane sweeps the compacted
// list reading each record by LDS broadcast.  Each lane accumulates only its
// own target's sums (gather form): no atomics, deterministic results.
//
// Mixed precision: positions are an integer cell plus an FP32 offset from the
// cell centre.  The displacement r_j - r_i along an axis is
//   fl32( fl32(o_j + (c_j - c_i) cs) - o_i )
// and r^2 = ((dx dx + dy dy) + dz dz) rounded after every operation, so the
// neighbour decision does not depend on how particles are grouped.  Densities
// enter as rho - rho0, which keeps the delta-SPH differences and the pressure
// accurate in FP32.  FP64: absolute positions, d = r_j - r_i, the same r^2.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "common.h"

namespace wcsph {

struct InteractArgs {
    const int4 *chunks;
    const DevScalars *sc;
    const uint32_t *keys;        // sorted cell id of every particle
    const uint32_t *cell_start;  // ncells + 1
    const void *v0, *v1, *v2;    // interaction view
    void *ax, *ay, *az, *drho, *mumax;
    unsigned long long *dt_min_bits;
    unsigned long long *pairs;   // running totals: fluid-fluid, fluid-boundary, boundary-fluid
    const uint32_t *id;          // original ids (neighbour statistics only)
    int32_t *st_nf, *st_nb;      // per-particle fluid / boundary neighbour counts
    uint32_t *st_hash;           // per-particle sum of id_hash(id_j) mod 2^32
    int nx, ny, nz;
    uint32_t nblocks;
    double cs, h, invh, r2max, eta2, Fm, alpha, kdelta, rho0, c0, gx, gy, gz;
    int delta_all;
};

__device__ __forceinline__ float sq_sum_f32(float dx, float dy, float dz) {
#pragma clang fp contract(off)
    float a = dx * dx;
    float b = dy * dy;
    float c = dz * dz;
    return (a + b) + c;
}

__device__ __forceinline__ double sq_sum_f64(double dx, double dy, double dz) {
#pragma clang fp contract(off)
    double a = dx * dx;
    double b = dy * dy;
    double c = dz * dz;
    return (a + b) + c;
}

template <class T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        T o = __shfl_xor(v, off, kWave);
        v = o < v ? o : v;
    }
    return v;
}

template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        T o = __shfl_xor(v, off, kWave);
        v = o > v ? o : v;
    }
    return v;
}

__device__ __forceinline__ uint64_t lanes_below() {
    uint32_t lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// 32-bit integer mixer (the finaliser of MurmurHash3): neighbour-set hashes
// are sums of id_hash over the set, so they do not depend on visit order.
__device__ __forceinline__ uint32_t id_hash(uint32_t v) {
    v ^= v >> 16;
    v *= 0x85ebca6bu;
    v ^= v >> 13;
    v *= 0xc2b2ae35u;
    v ^= v >> 16;
    return v;
}

// Adds the wave's pair counts to the running totals (one atomic per class).
__device__ __forceinline__ void add_pairs(unsigned long long *tot, uint32_t ff, uint32_t fb,
                                          uint32_t bf) {
    if (__lane_id() == 0) {
        if (ff) atomicAdd(&tot[0], (unsigned long long)ff);
        if (fb) atomicAdd(&tot[1], (unsigned long long)fb);
        if (bf) atomicAdd(&tot[2], (unsigned long long)bf);
    }
}

// Chunk handled by this block: consecutive chunks go to the same XCD (blocks
// are dealt round-robin to the 8 XCDs), so neighbouring chunks share L2.
__device__ __forceinline__ uint32_t xcd_chunk(uint32_t b, uint32_t nb) {
    const uint32_t per = nb / 8;  // nb is a multiple of 8
    return (b % 8) * per + b / 8;
}

// ------------------------------------------------------------ mixed FP32

template <bool kStats>
__global__ __launch_bounds__(kWave) void k_interact_mixed(InteractArgs a) {
    __shared__ float4 s0[kWave];  // {o_x, c_x, o_y + dy cs, o_z + dz cs}
    __shared__ float4 s1[kWave];  // {u_x, u_y, u_z, P}
    __shared__ float4 s2[kWave];  // {index bits, 1/rho, rho - rho0, +-c (- = boundary)}

    const uint32_t chunk = xcd_chunk(blockIdx.x, a.nblocks);
    if (chunk >= a.sc->nchunks) return;
    const int4 ch = a.chunks[chunk];
    const int cs0 = uni(ch.x), cs1 = uni(ch.y), row = uni(ch.z);
    const int cy = row % a.ny, cz = row / a.ny;
    const int lane = threadIdx.x;
    const int i = cs0 + lane;
    const bool act = i < cs1;
    const float4 *V0 = static_cast<const float4 *>(a.v0);
    const float4 *V1 = static_cast<const float4 *>(a.v1);
    const float2 *V2 = static_cast<const float2 *>(a.v2);
    const int rowbase = row * a.nx;
    const int cxa = uni((int)a.keys[cs0] - rowbase);
    const int cxb = uni((int)a.keys[cs1 - 1] - rowbase);
    const float csf = (float)a.cs;

    float4 ti0 = make_float4(0.f, 0.f, 0.f, 0.f), ti1 = ti0;
    float2 ti2 = make_float2(1.f, 1.f);
    int cix = cxa;
    if (act) {
        ti0 = V0[i];
        ti1 = V1[i];
        ti2 = V2[i];
        cix = (int)a.keys[i] - rowbase;
    }
    const float cixf = (float)cix;
    const bool fi = act && ti2.y > 0.f;
    // chunk bounding box in the frame of cell (cxa, cy, cz)
    const float bx = ti0.x + (float)(cix - cxa) * csf;
    float lox = wave_min(act ? bx : 3.0e38f), hix = wave_max(act ? bx : -3.0e38f);
    float loy = wave_min(act ? ti0.y : 3.0e38f), hiy = wave_max(act ? ti0.y : -3.0e38f);
    float loz = wave_min(act ? ti0.z : 3.0e38f), hiz = wave_max(act ? ti0.z : -3.0e38f);
    const bool any_fluid = __ballot(fi) != 0ull;
    // cull radius: 2h with a relative margin far above FP32 rounding
    const float cull2 = (float)(a.r2max * (1.0 + 1e-3)) + 1e-30f;
    const float r2max = (float)a.r2max;
    const float h = (float)a.h, invh = (float)a.invh, eta2 = (float)a.eta2;
    const float Fm = (float)a.Fm, alpha = (float)a.alpha, kdel = (float)a.kdelta;
    const float two_rho0 = (float)(2.0 * a.rho0);
    const bool dall = a.delta_all != 0;

    float sax = 0.f, say = 0.f, saz = 0.f, sdr = 0.f, mum = 0.f;
    const float oix = ti0.x, oiy = ti0.y, oiz = ti0.z, dri = ti0.w;
    const float uix = ti1.x, uiy = ti1.y, uiz = ti1.z, Pi = ti1.w;
    const float invri = ti2.x, ci = fabsf(ti2.y);
    const uint64_t below = lanes_below();
    const uint64_t fmask = __ballot(fi);
    uint32_t n_ff = 0, n_fb = 0, n_bf = 0;  // wave pair counts (scalar)
    int32_t st_f = 0, st_b = 0;
    uint32_t st_h = 0;

    for (int dz = -1; dz <= 1; ++dz) {
        const int czn = cz + dz;
        if (czn < 0 || czn >= a.nz) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            const int cyn = cy + dy;
            if (cyn < 0 || cyn >= a.ny) continue;
            const int nrow = czn * a.ny + cyn;
            const int nbase = nrow * a.nx;
            const int xlo = cxa - 1 < 0 ? 0 : cxa - 1;
            const int xhi = cxb + 1 >= a.nx ? a.nx - 1 : cxb + 1;
            const int js = uni((int)a.cell_start[nbase + xlo]);
            const int je = uni((int)a.cell_start[nbase + xhi + 1]);
            const float shy = (float)dy * csf, shz = (float)dz * csf;
            for (int jb = js; jb < je; jb += kWave) {
                const int j = jb + lane;
                bool keep = false;
                float4 c0 = make_float4(0.f, 0.f, 0.f, 0.f), c1 = c0;
                float2 c2 = make_float2(0.f, 0.f);
                float cjx = 0.f;
                if (j < je) {
                    c0 = V0[j];
                    c1 = V1[j];
                    c2 = V2[j];
                    const int cx = (int)a.keys[j] - nbase;
                    cjx = (float)cx;
                    const float qx = c0.x + (float)(cx - cxa) * csf;
                    const float qy = c0.y + shy, qz = c0.z + shz;
                    const float ex = fmaxf(fmaxf(lox - qx, qx - hix), 0.f);
                    const float ey = fmaxf(fmaxf(loy - qy, qy - hiy), 0.f);
                    const float ez = fmaxf(fmaxf(loz - qz, qz - hiz), 0.f);
                    keep = (ex * ex + ey * ey + ez * ez) <= cull2 && (any_fluid || c2.y > 0.f);
                }
                const uint64_t m = __ballot(keep);
                if (keep) {
                    const int slot = __popcll(m & below);
                    s0[slot] = make_float4(c0.x, cjx, c0.y + shy, c0.z + shz);
                    s1[slot] = c1;
                    s2[slot] = make_float4(__int_as_float(j), c2.x, c0.w, c2.y);
                }
                __syncthreads();
                const int cnt = __popcll(m);
                // partial sums per staged batch: the running sums see one
                // rounding per batch instead of one per pair
                float bax = 0.f, bay = 0.f, baz = 0.f, bdr = 0.f;
                for (int k = 0; k < cnt; ++k) {
                    const float4 r0 = s0[k];
                    const float4 r1 = s1[k];
                    const float4 r2 = s2[k];
                    const bool fj = r2.w > 0.f;
                    const float sx = fmaf(r0.y - cixf, csf, r0.x);
                    const float dx = sx - oix;
                    const float dy_ = r0.z - oiy;
                    const float dz_ = r0.w - oiz;
                    const float rr = sq_sum_f32(dx, dy_, dz_);
                    const bool in = act && rr < r2max && __float_as_int(r2.x) != i && (fi || fj);
                    const uint64_t inm = __ballot(in);
                    if (fj) {
                        n_ff += (uint32_t)__popcll(inm & fmask);
                        n_bf += (uint32_t)__popcll(inm & ~fmask);
                    } else {
                        n_fb += (uint32_t)__popcll(inm);
                    }
                    if (kStats && in) {
                        if (fj) ++st_f; else ++st_b;
                        st_h += id_hash(a.id[__float_as_int(r2.x)] & 0x7fffffffu);
                    }
                    if (in) {
                        const float q = __builtin_amdgcn_sqrtf(rr) * invh;
                        const float t = 1.f - 0.5f * q;
                        const float F = Fm * t * t * t;  // m * 5 w_D / h^2 * (1 - q/2)^3
                        const float vx = r1.x - uix, vy = r1.y - uiy, vz = r1.z - uiz;
                        const float vr = vx * dx + vy * dy_ + vz * dz_;
                        const float mu = h * vr * __builtin_amdgcn_rcpf(rr + eta2);
                        mum = fmaxf(mum, fabsf(mu));
                        bdr -= F * vr;  // m (u_i - u_j) . grad_i W_ij
                        if (fi) {
                            if (fj || dall) bdr += kdel * (r2.z - dri) * F * r2.y;
                            float visc = 0.f;
                            if (vr < 0.f)
                                visc = -alpha * (ci + fabsf(r2.w)) * mu *
                                       __builtin_amdgcn_rcpf(two_rho0 + dri + r2.z);
                            const float coef = ((Pi + r1.w) * invri * r2.y + visc) * F;
                            bax -= coef * dx;
                            bay -= coef * dy_;
                            baz -= coef * dz_;
                        }
                    }
                }
                sax += bax;
                say += bay;
                saz += baz;
                sdr += bdr;
                __syncthreads();
            }
        }
    }
    double bound = __longlong_as_double(0x7ff0000000000000ll);
    if (act) {
        float* oax = static_cast<float *>(a.ax);
        float* oay = static_cast<float *>(a.ay);
        float* oaz = static_cast<float *>(a.az);
        float fax = 0.f, fay = 0.f, faz = 0.f;
        if (fi) {
            fax = sax + (float)a.gx;
            fay = say + (float)a.gy;
            faz = saz + (float)a.gz;
        }
        oax[i] = fax;
        oay[i] = fay;
        oaz[i] = faz;
        static_cast<float *>(a.drho)[i] = sdr;
        static_cast<float *>(a.mumax)[i] = mum;
        bound = a.h / (a.c0 + (double)mum);
        if (fi) {
            const double am = sqrt((double)fax * fax + (double)fay * fay + (double)faz * faz);
            if (am > 0.0) bound = fmin(bound, sqrt(a.h / am));
        }
    }
    if (kStats && act) {
        a.st_nf[i] = st_f;
        a.st_nb[i] = st_b;
        a.st_hash[i] = st_h;
    }
    add_pairs(a.pairs, n_ff, n_fb, n_bf);
    bound = wave_min(bound);
    if (lane == 0)
        atomicMin(a.dt_min_bits, (unsigned long long)__double_as_longlong(bound));
}

// ------------------------------------------------------------------ FP64

template <bool kStats>
__global__ __launch_bounds__(kWave) void k_interact_fp64(InteractArgs a) {
    __shared__ double4 s0[kWave];  // {x, y, z, index}
    __shared__ double4 s1[kWave];  // {u_x, u_y, u_z, P}
    __shared__ double4 s2[kWave];  // {1/rho, rho, +-c, -}

    const uint32_t chunk = xcd_chunk(blockIdx.x, a.nblocks);
    if (chunk >= a.sc->nchunks) return;
    const int4 ch = a.chunks[chunk];
    const int cs0 = uni(ch.x), cs1 = uni(ch.y), row = uni(ch.z);
    const int cy = row % a.ny, cz = row / a.ny;
    const int lane = threadIdx.x;
    const int i = cs0 + lane;
    const bool act = i < cs1;
    const double4 *V0 = static_cast<const double4 *>(a.v0);
    const double4 *V1 = static_cast<const double4 *>(a.v1);
    const double2 *V2 = static_cast<const double2 *>(a.v2);
    const int rowbase = row * a.nx;
    const int cxa = uni((int)a.keys[cs0] - rowbase);
    const int cxb = uni((int)a.keys[cs1 - 1] - rowbase);

    double4 ti0 = make_double4(0, 0, 0, 1), ti1 = make_double4(0, 0, 0, 0);
    double2 ti2 = make_double2(1, 1);
    if (act) {
        ti0 = V0[i];
        ti1 = V1[i];
        ti2 = V2[i];
    }
    const bool fi = act && ti2.y > 0.0;
    double lox = wave_min(act ? ti0.x : 1e300), hix = wave_max(act ? ti0.x : -1e300);
    double loy = wave_min(act ? ti0.y : 1e300), hiy = wave_max(act ? ti0.y : -1e300);
    double loz = wave_min(act ? ti0.z : 1e300), hiz = wave_max(act ? ti0.z : -1e300);
    const bool any_fluid = __ballot(fi) != 0ull;
    const double cull2 = a.r2max * (1.0 + 1e-6);
    const bool dall = a.delta_all != 0;

    double sax = 0, say = 0, saz = 0, sdr = 0, mum = 0;
    const double xi = ti0.x, yi = ti0.y, zi = ti0.z, rhoi = ti0.w;
    const double uix = ti1.x, uiy = ti1.y, uiz = ti1.z, Pi = ti1.w;
    const double invri = ti2.x, ci = fabs(ti2.y);
    const uint64_t below = lanes_below();
    const uint64_t fmask = __ballot(fi);
    uint32_t n_ff = 0, n_fb = 0, n_bf = 0;  // wave pair counts (scalar)
    int32_t st_f = 0, st_b = 0;
    uint32_t st_h = 0;

    for (int dz = -1; dz <= 1; ++dz) {
        const int czn = cz + dz;
        if (czn < 0 || czn >= a.nz) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            const int cyn = cy + dy;
            if (cyn < 0 || cyn >= a.ny) continue;
            const int nbase = (czn * a.ny + cyn) * a.nx;
            const int xlo = cxa - 1 < 0 ? 0 : cxa - 1;
            const int xhi = cxb + 1 >= a.nx ? a.nx - 1 : cxb + 1;
            const int js = uni((int)a.cell_start[nbase + xlo]);
            const int je = uni((int)a.cell_start[nbase + xhi + 1]);
            for (int jb = js; jb < je; jb += kWave) {
                const int j = jb + lane;
                bool keep = false;
                double4 c0 = make_double4(0, 0, 0, 0), c1 = c0;
                double2 c2 = make_double2(0, 0);
                if (j < je) {
                    c0 = V0[j];
                    c1 = V1[j];
                    c2 = V2[j];
                    const double ex = fmax(fmax(lox - c0.x, c0.x - hix), 0.0);
                    const double ey = fmax(fmax(loy - c0.y, c0.y - hiy), 0.0);
                    const double ez = fmax(fmax(loz - c0.z, c0.z - hiz), 0.0);
                    keep = (ex * ex + ey * ey + ez * ez) <= cull2 && (any_fluid || c2.y > 0.0);
                }
                const uint64_t m = __ballot(keep);
                if (keep) {
                    const int slot = __popcll(m & below);
                    s0[slot] = make_double4(c0.x, c0.y, c0.z, (double)j);
                    s1[slot] = c1;
                    s2[slot] = make_double4(c2.x, c0.w, c2.y, 0.0);
                }
                __syncthreads();
                const int cnt = __popcll(m);
                for (int k = 0; k < cnt; ++k) {
                    const double4 r0 = s0[k];
                    const double4 r1 = s1[k];
                    const double4 r2 = s2[k];
                    const bool fj = r2.z > 0.0;
                    const double dx = r0.x - xi, dy_ = r0.y - yi, dz_ = r0.z - zi;
                    const double rr = sq_sum_f64(dx, dy_, dz_);
                    const bool in = act && rr < a.r2max && (int)r0.w != i && (fi || fj);
                    const uint64_t inm = __ballot(in);
                    if (fj) {
                        n_ff += (uint32_t)__popcll(inm & fmask);
                        n_bf += (uint32_t)__popcll(inm & ~fmask);
                    } else {
                        n_fb += (uint32_t)__popcll(inm);
                    }
                    if (kStats && in) {
                        if (fj) ++st_f; else ++st_b;
                        st_h += id_hash(a.id[(int)r0.w] & 0x7fffffffu);
                    }
                    if (in) {
                        const double q = sqrt(rr) * a.invh;
                        const double t = 1.0 - 0.5 * q;
                        const double F = a.Fm * t * t * t;
                        const double vx = r1.x - uix, vy = r1.y - uiy, vz = r1.z - uiz;
                        const double vr = vx * dx + vy * dy_ + vz * dz_;
                        const double mu = a.h * vr / (rr + a.eta2);
                        mum = fmax(mum, fabs(mu));
                        sdr -= F * vr;
                        if (fi) {
                            if (fj || dall) sdr += a.kdelta * (r2.y - rhoi) * F * r2.x;
                            double visc = 0.0;
                            if (vr < 0.0) visc = -a.alpha * (ci + fabs(r2.z)) * mu / (rhoi + r2.y);
                            const double coef = ((Pi + r1.w) * invri * r2.x + visc) * F;
                            sax -= coef * dx;
                            say -= coef * dy_;
                            saz -= coef * dz_;
                        }
                    }
                }
                __syncthreads();
            }
        }
    }
    double bound = __longlong_as_double(0x7ff0000000000000ll);
    if (act) {
        double fax = 0, fay = 0, faz = 0;
        if (fi) {
            fax = sax + a.gx;
            fay = say + a.gy;
            faz = saz + a.gz;
        }
        static_cast<double *>(a.ax)[i] = fax;
        static_cast<double *>(a.ay)[i] = fay;
        static_cast<double *>(a.az)[i] = faz;
        static_cast<double *>(a.drho)[i] = sdr;
        static_cast<double *>(a.mumax)[i] = mum;
        bound = a.h / (a.c0 + mum);
        if (fi) {
            const double am = sqrt(fax * fax + fay * fay + faz * faz);
            if (am > 0.0) bound = fmin(bound, sqrt(a.h / am));
        }
    }
    if (kStats && act) {
        a.st_nf[i] = st_f;
        a.st_nb[i] = st_b;
        a.st_hash[i] = st_h;
    }
    add_pairs(a.pairs, n_ff, n_fb, n_bf);
    bound = wave_min(bound);
    if (lane == 0)
        atomicMin(a.dt_min_bits, (unsigned long long)__double_as_longlong(bound));
}

int launch_interact(const sph_params &p, const sph_state &s, const Ws &w, hipStream_t st,
                    int32_t *st_nf, int32_t *st_nb, uint32_t *st_hash) {
    InteractArgs a;
    a.chunks = w.chunks();
    a.sc = w.scalars();
    a.keys = w.at<uint32_t>(w.L.sorted_keys);
    a.cell_start = w.cell_start();
    a.v0 = w.base + w.L.view0;
    a.v1 = w.base + w.L.view1;
    a.v2 = w.base + w.L.view2;
    const int64_t n = s.n;
    char *r = w.base + w.L.rates;
    const size_t e = w.L.rate_elem;
    a.ax = r;
    a.ay = r + e * n;
    a.az = r + 2 * e * n;
    a.drho = r + 3 * e * n;
    a.mumax = r + 4 * e * n;
    a.dt_min_bits = &w.scalars()->dt_min_bits;
    a.pairs = w.scalars()->pairs;
    a.id = s.id;
    a.st_nf = st_nf;
    a.st_nb = st_nb;
    a.st_hash = st_hash;
    const bool stats = st_nf != nullptr;
    a.nx = p.dims[0];
    a.ny = p.dims[1];
    a.nz = p.dims[2];
    const uint32_t nb = (uint32_t)((w.L.max_chunks + 7) / 8 * 8);
    a.nblocks = nb;
    a.cs = p.cell_size;
    a.h = p.h;
    a.invh = 1.0 / p.h;
    a.r2max = 4.0 * p.h * p.h;
    a.eta2 = p.eta2_coef * p.h * p.h;
    const double wd = 21.0 / (16.0 * M_PI * p.h * p.h * p.h);
    a.Fm = p.mass * 5.0 * wd / (p.h * p.h);
    a.alpha = p.alpha;
    a.kdelta = 2.0 * p.delta * p.h * p.c0;
    a.rho0 = p.rho0;
    a.c0 = p.c0;
    a.gx = p.g[0];
    a.gy = p.g[1];
    a.gz = p.g[2];
    a.delta_all = p.delta_pairs == SPH_DELTA_ALL;
    if (p.precision == SPH_MIXED) {
        if (stats)
            hipLaunchKernelGGL(k_interact_mixed<true>, dim3(nb), dim3(kWave), 0, st, a);
        else
            hipLaunchKernelGGL(k_interact_mixed<false>, dim3(nb), dim3(kWave), 0, st, a);
    } else {
        if (stats)
            hipLaunchKernelGGL(k_interact_fp64<true>, dim3(nb), dim3(kWave), 0, st, a);
        else
            hipLaunchKernelGGL(k_interact_fp64<false>, dim3(nb), dim3(kWave), 0, st, a);
    }
    return launch_check("interact");
}

// Copy the internal rates (FP32 or FP64, current order) to FP64 outputs.
template <class T>
__global__ void k_export(const T *__restrict__ r, int64_t n, double *ax, double *ay, double *az,
                         double *dr, double *mm) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    ax[i] = (double)r[i];
    ay[i] = (double)r[n + i];
    az[i] = (double)r[2 * n + i];
    dr[i] = (double)r[3 * n + i];
    if (mm) mm[i] = (double)r[4 * n + i];
}

int launch_export_rates(const sph_params &p, const Ws &w, int64_t n, double *ax, double *ay,
                        double *az, double *drho, double *mumax, hipStream_t st) {
    int blocks = (int)((n + 255) / 256);
    if (p.precision == SPH_MIXED)
        hipLaunchKernelGGL(k_export<float>, dim3(blocks), dim3(256), 0, st,
                           w.at<const float>(w.L.rates), n, ax, ay, az, drho, mumax);
    else
        hipLaunchKernelGGL(k_export<double>, dim3(blocks), dim3(256), 0, st,
                           w.at<const double>(w.L.rates), n, ax, ay, az, drho, mumax);
    return launch_check("export rates");
}

}  // namespace wcsph
