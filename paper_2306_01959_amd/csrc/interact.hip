// Pairwise WCSPH interaction (Section 2.2, eqs. sphu, pi, cpmu, sphw,
// sphrho, tait) and the per-particle time-step bound (eq. sphdt).
//
// Work decomposition.  A chunk is up to 64 consecutive sorted particles of
// one cell row (fixed cy, cz; cells are numbered x-fastest), one target per
// lane.  Its candidates are the nine stencil rows (cy+dy, cz+dz) over cells
// [cx_first - 1, cx_last + 1], each a contiguous range of the sorted arrays.
// A workgroup of kSplit waves (1, 3 or 9) owns a chunk; each wave takes 9 /
// kSplit of the rows, and the waves' partial sums are added in a fixed order
// at the end, so more waves cover the chip on small problems without changing
// results between runs.
//
// Per wave, candidates stream through in batches of 64: the next batch is
// loaded into registers while the current one is processed; a batch is
// culled against the chunk's bounding box (conservatively: 2h plus a relative
// margin), compacted into LDS with a ballot and a popcount, and every lane
// then sweeps the compacted records by LDS broadcast, accumulating only its
// own target's sums (gather form: no atomics, deterministic).  Quantities that
// depend on the candidate alone (P_j/rho_j, the delta-term factors) are
// computed once at staging instead of once per lane.
//
// Mixed precision: positions are an integer cell plus an FP32 offset from the
// cell centre.  The displacement r_j - r_i along an axis is
//   fl32( fl32(o_j + (c_j - c_i) cs) - o_i )
// and r^2 = ((dx dx + dy dy) + dz dz) rounded after every operation, so the
// neighbour decision does not depend on how particles are grouped.  Densities
// enter as rho - rho0, which keeps the delta-SPH differences and the pressure
// accurate in FP32; pair terms are summed per staged batch before they enter
// the running sums.  FP64: absolute positions, d = r_j - r_i, the same r^2.
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

// Orders one wave's LDS writes before its later reads (and reads before
// later overwrites) without involving the other waves of the workgroup.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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

// Chunk handled by this block: consecutive chunks go to the same XCD (blocks
// are dealt round-robin to the 8 XCDs), so neighbouring chunks share L2.
__device__ __forceinline__ uint32_t xcd_chunk(uint32_t b, uint32_t nb) {
    const uint32_t per = nb / 8;  // nb is a multiple of 8
    return (b % 8) * per + b / 8;
}

// Per-lane sums of one target.
template <class R>
struct Acc {
    R ax = 0, ay = 0, az = 0, dr = 0;
};

// Scalar (wave-uniform) pair counters and per-lane statistics.
struct Counters {
    uint32_t ff = 0, fb = 0, bf = 0;
    int32_t st_f = 0, st_b = 0;
    uint32_t st_h = 0;
};

__device__ __forceinline__ void count_pairs(Counters &cn, uint64_t inm, uint64_t fmask_bits,
                                            bool fj) {
    const uint32_t nin = (uint32_t)__popcll(inm);
    const uint32_t nfin = (uint32_t)__popcll(inm & fmask_bits);
    cn.ff += fj ? nfin : 0u;
    cn.bf += fj ? nin - nfin : 0u;
    cn.fb += fj ? 0u : nin;
}

// ================================================================ policies
//
// A policy supplies the target registers, the raw candidate registers, the
// LDS record (four vectors of 4) written at staging, and the pair term.

struct Mixed {
    using R = float;
    using V4 = float4;
    struct Target {
        float ox, oy, oz, cixf;  // offset from own cell centre, own cell x
        float ux, uy, uz;
        float P, invr;           // invr = 1/rho_i for fluid, 0 for boundary
        float dr;                // rho_i - rho0
        float rsum;              // 2 rho0 + (rho_i - rho0)
        float c;                 // |c_i|
        float nalpha;            // -alpha for fluid, 0 for boundary
        float fmask;             // 1 for fluid, 0 for boundary
        bool act, fi;
        int i;
    };
    struct Cand {
        float4 v0, v1;
        float2 v2;
        int cx;
        bool ok;
    };
    // frame for the chunk bounding box: cell (cxa, cy, cz)
    __device__ static Target target(const InteractArgs &a, int i, bool act, int rowbase, int cxa,
                                    float &bx, float &by, float &bz) {
        Target t{};
        t.act = act;
        t.i = i;
        float4 v0 = make_float4(0.f, 0.f, 0.f, 0.f), v1 = v0;
        float2 v2 = make_float2(1.f, 1.f);
        int cix = cxa;
        if (act) {
            v0 = static_cast<const float4 *>(a.v0)[i];
            v1 = static_cast<const float4 *>(a.v1)[i];
            v2 = static_cast<const float2 *>(a.v2)[i];
            cix = (int)a.keys[i] - rowbase;
        }
        t.fi = act && v2.y > 0.f;
        t.ox = v0.x;
        t.oy = v0.y;
        t.oz = v0.z;
        t.dr = v0.w;
        t.cixf = (float)cix;
        t.ux = v1.x;
        t.uy = v1.y;
        t.uz = v1.z;
        t.P = v1.w;
        t.invr = t.fi ? v2.x : 0.f;
        t.rsum = (float)(2.0 * a.rho0) + v0.w;
        t.c = fabsf(v2.y);
        t.nalpha = t.fi ? -(float)a.alpha : 0.f;
        t.fmask = t.fi ? 1.f : 0.f;
        const float csf = (float)a.cs;
        bx = v0.x + (float)(cix - cxa) * csf;
        by = v0.y;
        bz = v0.z;
        return t;
    }
    __device__ static void load(const InteractArgs &a, int j, int je, int nbase, Cand &c) {
        c.ok = j < je;
        if (c.ok) {
            c.v0 = static_cast<const float4 *>(a.v0)[j];
            c.v1 = static_cast<const float4 *>(a.v1)[j];
            c.v2 = static_cast<const float2 *>(a.v2)[j];
            c.cx = (int)a.keys[j] - nbase;
        } else {
            c.v0 = make_float4(0.f, 0.f, 0.f, 0.f);
            c.v1 = c.v0;
            c.v2 = make_float2(1.f, 1.f);
            c.cx = 0;
        }
    }
    // position of the candidate in the chunk frame, for culling only
    __device__ static void cull_pos(const InteractArgs &a, const Cand &c, int cxa, int dy, int dz,
                                    float &qx, float &qy, float &qz) {
        const float csf = (float)a.cs;
        qx = c.v0.x + (float)(c.cx - cxa) * csf;
        qy = c.v0.y + (float)dy * csf;
        qz = c.v0.z + (float)dz * csf;
    }
    __device__ static bool cand_fluid(const Cand &c) { return c.v2.y > 0.f; }
    // record: {o_x, c_x, o_y + dy cs, o_z + dz cs}, {u, P/rho}, {index bits,
    // 1/rho, (rho - rho0) B, B} with B = 2 delta h c0 / rho (0 when the pair
    // carries no delta term), {rho - rho0, +-c (- = boundary), -, -}
    __device__ static void stage(const InteractArgs &a, const Cand &c, int j, int dy, int dz,
                                 float4 *rec0, float4 *rec1, float4 *rec2, float4 *rec3) {
        const float csf = (float)a.cs;
        const float invr = c.v2.x;
        const bool fj = c.v2.y > 0.f;
        const float kd = (fj || a.delta_all) ? (float)a.kdelta : 0.f;
        const float B = kd * invr;
        *rec0 = make_float4(c.v0.x, (float)c.cx, c.v0.y + (float)dy * csf,
                            c.v0.z + (float)dz * csf);
        *rec1 = make_float4(c.v1.x, c.v1.y, c.v1.z, c.v1.w * invr);
        *rec2 = make_float4(__int_as_float(j), invr, c.v0.w * B, B);
        *rec3 = make_float4(c.v0.w, c.v2.y, 0.f, 0.f);
    }
    template <bool kStats>
    __device__ static void pair(const InteractArgs &a, const Target &t, const float4 &r0,
                                const float4 &r1, const float4 &r2, const float4 &r3,
                                uint64_t fmask_bits, Acc<float> &acc, float &mum, Counters &cn) {
        const float csf = (float)a.cs;
        const bool fj = uni(__float_as_int(r3.y)) > 0;  // record is wave-uniform
        const float sx = fmaf(r0.y - t.cixf, csf, r0.x);
        const float dx = sx - t.ox;
        const float dy = r0.z - t.oy;
        const float dz = r0.w - t.oz;
        const float rr = sq_sum_f32(dx, dy, dz);
        const int j = __float_as_int(r2.x);
        const bool in = t.act && rr < (float)a.r2max && j != t.i && (t.fi || fj);
        const uint64_t inm = __ballot(in);
        if (inm == 0) return;
        count_pairs(cn, inm, fmask_bits, fj);
        if (kStats && in) {
            if (fj)
                ++cn.st_f;
            else
                ++cn.st_b;
            cn.st_h += id_hash(a.id[j] & 0x7fffffffu);
        }
        const float r = __builtin_amdgcn_sqrtf(rr);
        const float q2 = fmaf(r, -0.5f * (float)a.invh, 1.f);  // 1 - q/2
        const float F = in ? (float)a.Fm * q2 * q2 * q2 : 0.f;   // m 5 w_D/h^2 (1-q/2)^3
        const float vx = r1.x - t.ux, vy = r1.y - t.uy, vz = r1.z - t.uz;
        const float vr = vx * dx + vy * dy + vz * dz;               // u_ij . r_ij
        const float mu = (float)a.h * vr * __builtin_amdgcn_rcpf(rr + (float)a.eta2);
        mum = in ? fmaxf(mum, fabsf(mu)) : mum;
        acc.dr -= F * vr;                                     // m (u_i - u_j) . grad_i W_ij
        acc.dr += fmaf(-t.dr, r2.w, r2.z) * (F * t.fmask);    // delta term
        const float visc = vr < 0.f ? t.nalpha * (t.c + fabsf(r3.y)) * mu *
                                          __builtin_amdgcn_rcpf(t.rsum + r3.x)
                                    : 0.f;
        const float s = (fmaf(t.P, r2.y, r1.w) * t.invr + visc) * F;
        acc.ax -= s * dx;
        acc.ay -= s * dy;
        acc.az -= s * dz;
    }
    __device__ static void store(const InteractArgs &a, int i, const Target &t, float ax, float ay,
                                 float az, float dr, float mum, double &bound) {
        float fax = 0.f, fay = 0.f, faz = 0.f;
        if (t.fi) {
            fax = ax + (float)a.gx;
            fay = ay + (float)a.gy;
            faz = az + (float)a.gz;
        }
        static_cast<float *>(a.ax)[i] = fax;
        static_cast<float *>(a.ay)[i] = fay;
        static_cast<float *>(a.az)[i] = faz;
        static_cast<float *>(a.drho)[i] = dr;
        static_cast<float *>(a.mumax)[i] = mum;
        bound = a.h / (a.c0 + (double)mum);
        if (t.fi) {
            const double am = sqrt((double)fax * fax + (double)fay * fay + (double)faz * faz);
            if (am > 0.0) bound = fmin(bound, sqrt(a.h / am));
        }
    }
};

struct Fp64 {
    using R = double;
    using V4 = double4;
    struct Target {
        double x, y, z, ux, uy, uz, P, invr, rho, c, nalpha, fmask;
        bool act, fi;
        int i;
    };
    struct Cand {
        double4 v0, v1;
        double2 v2;
        bool ok;
    };
    __device__ static Target target(const InteractArgs &a, int i, bool act, int rowbase, int cxa,
                                    double &bx, double &by, double &bz) {
        (void)rowbase;
        (void)cxa;
        Target t{};
        t.act = act;
        t.i = i;
        double4 v0 = make_double4(0, 0, 0, 1), v1 = make_double4(0, 0, 0, 0);
        double2 v2 = make_double2(1, 1);
        if (act) {
            v0 = static_cast<const double4 *>(a.v0)[i];
            v1 = static_cast<const double4 *>(a.v1)[i];
            v2 = static_cast<const double2 *>(a.v2)[i];
        }
        t.fi = act && v2.y > 0.0;
        t.x = v0.x;
        t.y = v0.y;
        t.z = v0.z;
        t.rho = v0.w;
        t.ux = v1.x;
        t.uy = v1.y;
        t.uz = v1.z;
        t.P = v1.w;
        t.invr = t.fi ? v2.x : 0.0;
        t.c = fabs(v2.y);
        t.nalpha = t.fi ? -a.alpha : 0.0;
        t.fmask = t.fi ? 1.0 : 0.0;
        bx = v0.x;
        by = v0.y;
        bz = v0.z;
        return t;
    }
    __device__ static void load(const InteractArgs &a, int j, int je, int nbase, Cand &c) {
        (void)nbase;
        c.ok = j < je;
        if (c.ok) {
            c.v0 = static_cast<const double4 *>(a.v0)[j];
            c.v1 = static_cast<const double4 *>(a.v1)[j];
            c.v2 = static_cast<const double2 *>(a.v2)[j];
        } else {
            c.v0 = make_double4(0, 0, 0, 1);
            c.v1 = make_double4(0, 0, 0, 0);
            c.v2 = make_double2(1, 1);
        }
    }
    __device__ static void cull_pos(const InteractArgs &a, const Cand &c, int cxa, int dy, int dz,
                                    double &qx, double &qy, double &qz) {
        (void)a;
        (void)cxa;
        (void)dy;
        (void)dz;
        qx = c.v0.x;
        qy = c.v0.y;
        qz = c.v0.z;
    }
    __device__ static bool cand_fluid(const Cand &c) { return c.v2.y > 0.0; }
    // record: {x, y, z, index}, {u, P/rho}, {1/rho, B, rho, +-c}, unused
    __device__ static void stage(const InteractArgs &a, const Cand &c, int j, int dy, int dz,
                                 double4 *rec0, double4 *rec1, double4 *rec2, double4 *rec3) {
        (void)dy;
        (void)dz;
        (void)rec3;
        const double invr = c.v2.x;
        const bool fj = c.v2.y > 0.0;
        const double B = (fj || a.delta_all) ? a.kdelta * invr : 0.0;
        *rec0 = make_double4(c.v0.x, c.v0.y, c.v0.z, (double)j);
        *rec1 = make_double4(c.v1.x, c.v1.y, c.v1.z, c.v1.w * invr);
        *rec2 = make_double4(invr, B, c.v0.w, c.v2.y);
    }
    template <bool kStats>
    __device__ static void pair(const InteractArgs &a, const Target &t, const double4 &r0,
                                const double4 &r1, const double4 &r2, const double4 &r3,
                                uint64_t fmask_bits, Acc<double> &acc, double &mum, Counters &cn) {
        (void)r3;
        const bool fj = uni(__double2hiint(r2.w)) > 0;  // record is wave-uniform
        const double dx = r0.x - t.x, dy = r0.y - t.y, dz = r0.z - t.z;
        const double rr = sq_sum_f64(dx, dy, dz);
        const int j = (int)r0.w;
        const bool in = t.act && rr < a.r2max && j != t.i && (t.fi || fj);
        const uint64_t inm = __ballot(in);
        if (inm == 0) return;
        count_pairs(cn, inm, fmask_bits, fj);
        if (kStats && in) {
            if (fj)
                ++cn.st_f;
            else
                ++cn.st_b;
            cn.st_h += id_hash(a.id[j] & 0x7fffffffu);
        }
        const double q2 = 1.0 - 0.5 * (sqrt(rr) * a.invh);
        const double F = in ? a.Fm * q2 * q2 * q2 : 0.0;
        const double vx = r1.x - t.ux, vy = r1.y - t.uy, vz = r1.z - t.uz;
        const double vr = vx * dx + vy * dy + vz * dz;
        const double mu = a.h * vr / (rr + a.eta2);
        mum = in ? fmax(mum, fabs(mu)) : mum;
        acc.dr -= F * vr;
        acc.dr += (r2.z - t.rho) * r2.y * (F * t.fmask);
        const double visc = vr < 0.0 ? t.nalpha * (t.c + fabs(r2.w)) * mu / (t.rho + r2.z) : 0.0;
        const double s = (fma(t.P, r2.x, r1.w) * t.invr + visc) * F;
        acc.ax -= s * dx;
        acc.ay -= s * dy;
        acc.az -= s * dz;
    }
    __device__ static void store(const InteractArgs &a, int i, const Target &t, double ax,
                                 double ay, double az, double dr, double mum, double &bound) {
        double fax = 0, fay = 0, faz = 0;
        if (t.fi) {
            fax = ax + a.gx;
            fay = ay + a.gy;
            faz = az + a.gz;
        }
        static_cast<double *>(a.ax)[i] = fax;
        static_cast<double *>(a.ay)[i] = fay;
        static_cast<double *>(a.az)[i] = faz;
        static_cast<double *>(a.drho)[i] = dr;
        static_cast<double *>(a.mumax)[i] = mum;
        bound = a.h / (a.c0 + mum);
        if (t.fi) {
            const double am = sqrt(fax * fax + fay * fay + faz * faz);
            if (am > 0.0) bound = fmin(bound, sqrt(a.h / am));
        }
    }
};

// ================================================================ skeleton

template <class P, int kSplit, bool kStats>
__global__ __launch_bounds__(kWave *kSplit) void k_interact(InteractArgs a) {
    using R = typename P::R;
    using V4 = typename P::V4;
    constexpr int kRows = 9 / kSplit;
    // per-wave staging; after its loop a wave reuses its own region for the
    // cross-wave reduction (5 sums of R and 3 int32 per lane fit in 4 V4)
    __shared__ V4 stg[kSplit][4][kWave];
    __shared__ int4 rows[kSplit][kRows];
    static_assert(sizeof(R) * 5 + 4 * 3 <= sizeof(V4) * 4, "reduction fits the staging region");

    const int w = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const uint32_t chunk = xcd_chunk(blockIdx.x, a.nblocks);
    if (chunk >= a.sc->nchunks) return;  // uniform over the workgroup
    const int4 ch = a.chunks[chunk];
    const int cs0 = uni(ch.x), cs1 = uni(ch.y), row = uni(ch.z);
    const int cy = row % a.ny, cz = row / a.ny;
    const int i = cs0 + lane;
    const bool act = i < cs1;
    const int rowbase = row * a.nx;
    const int cxa = uni((int)a.keys[cs0] - rowbase);
    const int cxb = uni((int)a.keys[cs1 - 1] - rowbase);

    R bx, by, bz;
    const typename P::Target t = P::target(a, i, act, rowbase, cxa, bx, by, bz);
    const R big = (R)3.0e38f;
    const R lox = wave_min(act ? bx : big), hix = wave_max(act ? bx : -big);
    const R loy = wave_min(act ? by : big), hiy = wave_max(act ? by : -big);
    const R loz = wave_min(act ? bz : big), hiz = wave_max(act ? bz : -big);
    const uint64_t fmask_bits = __ballot(t.fi);
    const bool any_fluid = fmask_bits != 0ull;
    const R cull2 = (R)(a.r2max * (1.0 + 1e-3));
    const uint64_t below = lanes_below();

    // this wave's stencil rows: {first, end, row base cell, (dy+1) | (dz+1) << 2}
    if (lane < kRows) {
        const int rr = w * kRows + lane;
        const int dz = rr / 3 - 1, dy = rr % 3 - 1;
        const int czn = cz + dz, cyn = cy + dy;
        int js = 0, je = 0, nbase = 0;
        if (czn >= 0 && czn < a.nz && cyn >= 0 && cyn < a.ny) {
            nbase = (czn * a.ny + cyn) * a.nx;
            const int xlo = cxa - 1 < 0 ? 0 : cxa - 1;
            const int xhi = cxb + 1 >= a.nx ? a.nx - 1 : cxb + 1;
            js = (int)a.cell_start[nbase + xlo];
            je = (int)a.cell_start[nbase + xhi + 1];
        }
        rows[w][lane] = make_int4(js, je, nbase, (dy + 1) | ((dz + 1) << 2));
    }
    wave_sync();

    auto next_row = [&](int q) {
        while (q < kRows && rows[w][q].x >= rows[w][q].y) ++q;
        return q;
    };

    Acc<R> sum;
    R mum = 0;
    Counters cn;
    int q = uni(next_row(0));
    int jb = q < kRows ? uni(rows[w][q].x) : 0;
    typename P::Cand cur, nxt;
    if (q < kRows) P::load(a, jb + lane, rows[w][q].y, rows[w][q].z, cur);
    while (q < kRows) {
        const int4 rq = rows[w][q];
        const int dy = (rq.w & 3) - 1, dz = (rq.w >> 2) - 1;
        int q2 = q, jb2 = jb + kWave;
        if (jb2 >= rq.y) {
            q2 = uni(next_row(q + 1));
            jb2 = q2 < kRows ? uni(rows[w][q2].x) : 0;
        }
        if (q2 < kRows) P::load(a, jb2 + lane, rows[w][q2].y, rows[w][q2].z, nxt);

        // cull against the chunk box, compact the survivors into LDS
        bool keep = false;
        if (cur.ok) {
            R qx, qy, qz;
            P::cull_pos(a, cur, cxa, dy, dz, qx, qy, qz);
            const R ex = fmax(fmax(lox - qx, qx - hix), (R)0);
            const R ey = fmax(fmax(loy - qy, qy - hiy), (R)0);
            const R ez = fmax(fmax(loz - qz, qz - hiz), (R)0);
            keep = (ex * ex + ey * ey + ez * ez) <= cull2 && (any_fluid || P::cand_fluid(cur));
        }
        const uint64_t m = __ballot(keep);
        if (keep) {
            const int slot = __popcll(m & below);
            P::stage(a, cur, jb + lane, dy, dz, &stg[w][0][slot], &stg[w][1][slot],
                     &stg[w][2][slot], &stg[w][3][slot]);
        }
        wave_sync();
        const int cnt = __popcll(m);
        Acc<R> b;  // this batch's partial sums
        if (cnt > 0) {
            V4 n0 = stg[w][0][0], n1 = stg[w][1][0], n2 = stg[w][2][0], n3 = stg[w][3][0];
            for (int k = 0; k < cnt; ++k) {
                const V4 r0 = n0, r1 = n1, r2 = n2, r3 = n3;
                if (k + 1 < cnt) {
                    n0 = stg[w][0][k + 1];
                    n1 = stg[w][1][k + 1];
                    n2 = stg[w][2][k + 1];
                    n3 = stg[w][3][k + 1];
                }
                P::template pair<kStats>(a, t, r0, r1, r2, r3, fmask_bits, b, mum, cn);
            }
        }
        sum.ax += b.ax;
        sum.ay += b.ay;
        sum.az += b.az;
        sum.dr += b.dr;
        wave_sync();
        cur = nxt;
        q = q2;
        jb = jb2;
    }

    // pair totals: integer atomics, order does not matter
    if (lane == 0) {
        if (cn.ff) atomicAdd(&a.pairs[0], (unsigned long long)cn.ff);
        if (cn.fb) atomicAdd(&a.pairs[1], (unsigned long long)cn.fb);
        if (cn.bf) atomicAdd(&a.pairs[2], (unsigned long long)cn.bf);
    }
    if constexpr (kSplit > 1) {
        auto red = [&](int wave, int f) -> R & {
            return reinterpret_cast<R *>(&stg[wave][0][0])[f * kWave + lane];
        };
        auto redi = [&](int wave, int f) -> int32_t & {
            return reinterpret_cast<int32_t *>(reinterpret_cast<R *>(&stg[wave][0][0]) +
                                               5 * kWave)[f * kWave + lane];
        };
        red(w, 0) = sum.ax;
        red(w, 1) = sum.ay;
        red(w, 2) = sum.az;
        red(w, 3) = sum.dr;
        red(w, 4) = mum;
        if constexpr (kStats) {
            redi(w, 0) = cn.st_f;
            redi(w, 1) = cn.st_b;
            redi(w, 2) = (int32_t)cn.st_h;
        }
        __syncthreads();
        if (w != 0) return;
        // fixed summation order over the waves
        sum.ax = red(0, 0);
        sum.ay = red(0, 1);
        sum.az = red(0, 2);
        sum.dr = red(0, 3);
        mum = red(0, 4);
        for (int k = 1; k < kSplit; ++k) {
            sum.ax += red(k, 0);
            sum.ay += red(k, 1);
            sum.az += red(k, 2);
            sum.dr += red(k, 3);
            mum = red(k, 4) > mum ? red(k, 4) : mum;
            if constexpr (kStats) {
                cn.st_f += redi(k, 0);
                cn.st_b += redi(k, 1);
                cn.st_h += (uint32_t)redi(k, 2);
            }
        }
    }
    double bound = __longlong_as_double(0x7ff0000000000000ll);
    if (act) {
        P::store(a, i, t, sum.ax, sum.ay, sum.az, sum.dr, mum, bound);
        if constexpr (kStats) {
            a.st_nf[i] = cn.st_f;
            a.st_nb[i] = cn.st_b;
            a.st_hash[i] = cn.st_h;
        }
    }
    bound = wave_min(bound);
    if (lane == 0) atomicMin(a.dt_min_bits, (unsigned long long)__double_as_longlong(bound));
}

// ================================================================ launch

static int g_split[2] = {0, 0};  // 0 = automatic, else 1, 3 or 9 (per precision)

int set_split(int precision, int split) {
    if (precision != SPH_FP64 && precision != SPH_MIXED) return -1;
    if (split != 0 && split != 1 && split != 3 && split != 9) return -1;
    g_split[precision] = split;
    return 0;
}

int split_for(const sph_params &p, int64_t max_chunks) {
    const int s = g_split[p.precision == SPH_MIXED ? SPH_MIXED : SPH_FP64];
    if (s) return s;
    // enough waves to fill 256 CUs x 4 SIMDs several times over
    if (max_chunks < 2048) return 9;
    if (max_chunks < 16384) return 3;
    return 1;
}

template <class P, bool kStats>
static void launch_split(int split, uint32_t nb, const InteractArgs &a, hipStream_t st) {
    switch (split) {
    case 9:
        hipLaunchKernelGGL((k_interact<P, 9, kStats>), dim3(nb), dim3(kWave * 9), 0, st, a);
        break;
    case 3:
        hipLaunchKernelGGL((k_interact<P, 3, kStats>), dim3(nb), dim3(kWave * 3), 0, st, a);
        break;
    default:
        hipLaunchKernelGGL((k_interact<P, 1, kStats>), dim3(nb), dim3(kWave), 0, st, a);
        break;
    }
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
    const int split = split_for(p, w.L.max_chunks);
    if (p.precision == SPH_MIXED) {
        if (stats)
            launch_split<Mixed, true>(split, nb, a, st);
        else
            launch_split<Mixed, false>(split, nb, a, st);
    } else {
        if (stats)
            launch_split<Fp64, true>(split, nb, a, st);
        else
            launch_split<Fp64, false>(split, nb, a, st);
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
