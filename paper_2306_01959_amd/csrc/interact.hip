// Pairwise WCSPH interaction (Section 2.2, eqs. sphu, pi, cpmu, sphw,
// sphrho, tait) and the per-particle time-step bound (eq. sphdt).
//
// Work decomposition.  Particles are sorted by class (fluid before
// boundary), then cell row (fixed cy, cz), then cell x.  A chunk is up to 64 consecutive sorted
// particles of one half-row (the fluid or the boundary particles of a row),
// so it is all fluid or all boundary.  Its candidates are the nine stencil
// rows (cy+dy, cz+dz) over cells [cx_first - 1, cx_last + 1], each split
// into its fluid and its boundary half: eighteen contiguous ranges of the
// sorted arrays, of which a boundary chunk takes the nine fluid ones only.  A
// workgroup of kSplit waves (1, 3 or 9) owns a chunk; each wave takes
// 9 / kSplit of the stencil rows, and the waves' partial sums are added in a
// fixed order at the end.
//
// Per wave, candidates stream through in batches of 64: the next batch is
// loaded into registers while the current one is processed; a batch is
// culled against the chunk's bounding box (conservatively: 2h plus a relative
// margin) and compacted into LDS with a ballot and a popcount.  The chunk's
// targets are split into groups of kT consecutive particles (64 / kT groups),
// each with its own bounding box; every group keeps the staged records that
// can reach it (one ballot per group).  Lane l then works on target
// (l mod kT) of a group and on every (64 / kT)-th of that group's records, so
// a wave evaluates 64 (target, record) pairs per step; small groups are
// compact, which raises the share of evaluated pairs that lie inside the 2h
// support.  Each lane accumulates per group; at the end the lanes that share
// a target are summed with a fixed shuffle tree (gather form: no atomics,
// deterministic).  Candidate-only quantities (P_j/rho_j, the delta-term
// factors) are computed once at staging; factors common to all of a target's
// pairs (m 5 w_D / h^2 of the gradient, h of mu) are applied to its sums once,
// in store().
//
// Mixed precision: positions are an integer cell plus an FP32 offset from the
// cell centre.  The displacement r_j - r_i along an axis is
//   fl32( fl32(o_j + (c_j - c_i) cs) - o_i )
// and r^2 = ((dx dx + dy dy) + dz dz) rounded after every operation, so the
// neighbour decision does not depend on how particles are grouped.  Densities
// enter as rho - rho0, which keeps the delta-SPH differences and the pressure
// accurate in FP32.  FP64: absolute positions, d = r_j - r_i, the same r^2.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "common.h"
#include "update.h"

namespace wcsph {

struct InteractArgs {
    const int4 *chunks;
    DevScalars *sc;
    InstState *ist;
    Insts I;
    const uint32_t *keys;        // sorted keys (cell key, sub-cell bits)
    const uint32_t *cell_start;  // first sorted position of every key, 2 ncells + 1
    const void *v0, *v1, *v2;    // interaction view
    void *ax, *ay, *az, *drho, *mumax;
    ChunkOut *cout;              // per chunk: time-step bound and pair counts
    const uint32_t *id;          // original ids (neighbour statistics only)
    int32_t *st_nf, *st_nb;      // per-particle fluid / boundary neighbour counts
    uint32_t *st_hash;           // per-particle sum of id_hash(id_j) mod 2^32
    StateArrays state;           // fused update: the state to advance
    long long step;              // fused update: step index (selects the Euler reset)
    uint32_t xcd_run;            // chunks per XCD run (1: workgroups in chunk order)
    // fused update that writes the next sort's keys: with hist, also the
    // digit counts (from bit hist_shift) of its first pass per sort tile
    // (tiles of 2^tile_log2 positions; the counts start at zero)
    uint32_t *hist;
    int hist_shift, ntiles, tile_log2;
};

// Adds the keys of a wave's targets (one per lane, consecutive positions
// `it`) to the next sort's first-pass digit counts: equal (digit, tile) come
// in runs of consecutive lanes (nearly sorted keys), one atomic per run.  All
// lanes of the wave call it.
__device__ __forceinline__ void count_next_digit(const InteractArgs &a, bool act, int it,
                                                 uint32_t key) {
    const uint32_t slot =
        act ? ((key >> a.hist_shift) & (kRadix - 1)) * (uint32_t)a.ntiles +
                  ((uint32_t)it >> a.tile_log2)
            : 0xffffffffu;
    const uint64_t starts = run_starts(slot);
    if (act && ((starts >> __lane_id()) & 1ull)) atomicAdd(&a.hist[slot], run_length(starts));
}

// r^2 of the mixed path's neighbour predicate: fma(dz, dz, fma(dy, dy, dx dx)),
// each operation rounded once (three instructions; the FP32 brute force of
// the tests takes the same steps)
__device__ __forceinline__ float sq_sum_f32(float dx, float dy, float dz) {
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

__device__ __forceinline__ double sq_sum_f64(double dx, double dy, double dz) {
#pragma clang fp contract(off)
    double a = dx * dx;
    double b = dy * dy;
    double c = dz * dz;
    return (a + b) + c;
}

// min / max over aligned groups of `width` lanes (width a power of 2)
template <class T>
__device__ __forceinline__ T group_min(T v, int width) {
    for (int off = 1; off < width; off <<= 1) {
        T o = __shfl_xor(v, off, kWave);
        v = o < v ? o : v;
    }
    return v;
}

template <class T>
__device__ __forceinline__ T group_max(T v, int width) {
    for (int off = 1; off < width; off <<= 1) {
        T o = __shfl_xor(v, off, kWave);
        v = o > v ? o : v;
    }
    return v;
}

// Lanes below this one among those set in m (the hardware lane-rank count).
__device__ __forceinline__ int rank_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
// wave-uniform floating values (e.g. a wave-wide min) kept in scalar registers
__device__ __forceinline__ float uni(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uni(double v) {
    const long long b = __double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// max(a, |b|) for a >= 0 in one instruction (the absolute value is an input
// modifier of v_max_f32; written out because the compiler would first quiet
// possible signalling NaNs); a NaN b is dropped, as IEEE maxNum does
__device__ __forceinline__ float max_abs(float a, float b) {
    float r;
    asm("v_max_f32 %0, %1, |%2|" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// max of two non-negative floats: their bit patterns order like integers (one
// integer max, where fmaxf first quiets possible signalling NaNs)
__device__ __forceinline__ float max_nonneg(float a, float b) {
    return __int_as_float(max(__float_as_int(a), __float_as_int(b)));
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

// Per-lane sums of one (target, record subset).
template <class R>
struct Acc {
    R ax = 0, ay = 0, az = 0, dr = 0, mu = 0;
};

// Wave-uniform pair counters, and per-lane neighbour statistics of a group.
// Target classes a pair body may be specialised for: a chunk is one
// half-row, so all its targets are fluid or all boundary.
constexpr int kAnyTargets = 0, kFluidTargets = 1, kBoundaryTargets = 2;

// Pair counts, per lane: the (target, record) pairs inside the support.  A
// chunk's targets are all fluid or all boundary (one half-row), and a
// boundary chunk stages fluid records only.  A fluid chunk's count (which
// includes each target's pair with itself, r = 0, unless the pair body
// excludes it) is fluid-fluid + fluid-boundary; a boundary chunk's is
// boundary-fluid, and fluid-boundary equals it because the neighbour relation
// is symmetric (exactly in FP64; in mixed precision up to pairs within one
// FP32 rounding of 2h).  The record keeps {FF + FB, 0, BF}; the diagnostics
// split them.
struct Counters {
    uint32_t in = 0;
    // wave total (every lane of the wave calls it; uniform result)
    __device__ __forceinline__ uint32_t total() const {
        uint32_t a = in;
        for (int off = 1; off < kWave; off <<= 1) a += __shfl_xor(a, off, kWave);
        return a;
    }
};
struct Stats {
    int32_t f = 0, b = 0;
    uint32_t h = 0;
};

// ================================================================ policies
//
// A policy supplies the target record (three vectors of 4 in LDS), the raw
// candidate registers, the candidate record (four vectors of 4 in LDS)
// written at staging, and the pair term.

struct Mixed {
    using R = float;
    using V4 = float4;
    static constexpr bool kMixed = true;
    // target: {o_x, o_y, o_z, own cell x}, {u, P}, {1/rho (0 for boundary),
    // rho - rho0, -alpha |c|, 2 rho0 + (rho - rho0) in FP32}
    struct T {
        float4 a, b, c;
        __device__ bool fluid() const { return c.x > 0.f; }
    };
    // view: v0 {o_x, o_y, o_z, u_x}, v1 {u_y, u_z}, v2 {rho - rho0, P, 1/rho,
    // +-c}; only v2 changes for a fixed wall's particle
    struct Cand {
        float4 v0;
        float2 v1;
        float4 v2;
        uint32_t key;  // global cell (raw: nothing is computed from a load
                       // before it is needed, so the next batch's loads stay
                       // in flight while the current batch is processed)
        bool ok;
    };
    __device__ static void target(const InteractArgs &a, const Inst &ip, int i, bool act, int rowbase, int cxa,
                                  V4 &t0, V4 &t1, V4 &t2, float &bx, float &by, float &bz,
                                  bool &fi) {
        // an absent target sits far away (+1e15 m): no record is within its
        // support, not even a sentinel (which sits at -1e15 m)
        float4 v0 = make_float4(1e15f, 1e15f, 1e15f, 0.f), v2 = make_float4(0.f, 0.f, 1.f, 1.f);
        float2 v1 = make_float2(0.f, 0.f);
        int cix = cxa;
        if (act) {
            v0 = static_cast<const float4 *>(a.v0)[i];
            v1 = static_cast<const float2 *>(a.v1)[i];
            v2 = static_cast<const float4 *>(a.v2)[i];
            cix = (int)key_cell(a.keys[i]) - rowbase;
        }
        fi = act && v2.w > 0.f;
        t0 = make_float4(v0.x, v0.y, v0.z, (float)cix);
        t1 = make_float4(v0.w, v1.x, v1.y, v2.y);
        t2 = make_float4(fi ? v2.z : 0.f, v2.x, -(float)(ip.alpha * ip.h) * fabsf(v2.w),
                         (float)(2.0 * ip.rho0) + v2.x);
        const float csf = (float)ip.cs;
        bx = v0.x + (float)(cix - cxa) * csf;
        by = v0.y;
        bz = v0.z;
    }
    // Loads candidate j (< je), or for j >= je particle 0 with ok = false:
    // no branch around the loads, so the compiler can count them exactly
    // and wait for the current batch only.
    __device__ static void load(const InteractArgs &a, const Inst &ip, int j, int je, Cand &c) {
        c.ok = j < je;
        const int jj = c.ok ? j : 0;
        c.v0 = static_cast<const float4 *>(a.v0)[jj];
        c.v1 = static_cast<const float2 *>(a.v1)[jj];
        c.v2 = static_cast<const float4 *>(a.v2)[jj];
        c.key = key_cell(a.keys[jj]);
    }
    // position of a candidate in the chunk frame (cell cxa of the chunk's
    // row), for culling only; nbase = key of cell x = 0 of its half-row
    __device__ static void cull_pos(const InteractArgs &a, const Inst &ip, const Cand &c, int nbase,
                                    int cxa, int dy, int dz, float &qx, float &qy, float &qz) {
        const float csf = (float)ip.cs;
        qx = c.v0.x + (float)((int)c.key - nbase - cxa) * csf;
        qy = c.v0.y + (float)dy * csf;
        qz = c.v0.z + (float)dz * csf;
    }
    __device__ static void rec_pos(const InteractArgs &a, const Inst &ip, const float4 &r0, int cxa, float &qx,
                                   float &qy, float &qz) {
        qx = r0.x + (r0.y - (float)cxa) * (float)ip.cs;
        qy = r0.z;
        qz = r0.w;
    }
    __device__ static bool cand_fluid(const Cand &c) { return c.v2.w > 0.f; }
    __device__ static bool rec_fluid(const float4 &r3) { return r3.y > 0.f; }
    // a record that lies outside every target's support (at -1e15 m; every
    // term stays finite and is zeroed through F)
    __device__ static void sentinel(float4 *rec0, float4 *rec1, float4 *rec2, float4 *rec3) {
        *rec0 = make_float4(-1e15f, 0.f, -1e15f, -1e15f);
        *rec1 = make_float4(0.f, 0.f, 0.f, 0.f);
        *rec2 = *rec1;
        *rec3 = *rec1;
    }
    // record: {o_x, c_x, o_y + dy cs, o_z + dz cs}, {u, P/rho}, {rho - rho0,
    // 1/rho, (rho - rho0) B, B} with B = 2 delta h c0 / rho (0 when the pair
    // carries no delta term), {-alpha h |c|, +-c (- = boundary), index bits, -}
    // (the fluid pair body reads all of the first three and one value of the
    // fourth)
    __device__ static void stage(const InteractArgs &a, const Inst &ip, const Cand &c, int nbase,
                                 int j, int dy, int dz, float4 *rec0, float4 *rec1, float4 *rec2,
                                 float4 *rec3) {
        const float csf = (float)ip.cs;
        const float invr = c.v2.z;
        const bool fj = c.v2.w > 0.f;
        const float kd = (fj || ip.delta_all) ? (float)ip.kdelta : 0.f;
        const float B = kd * invr;
        *rec0 = make_float4(c.v0.x, (float)((int)c.key - nbase), c.v0.y + (float)dy * csf,
                            c.v0.z + (float)dz * csf);
        *rec1 = make_float4(c.v0.w, c.v1.x, c.v1.y, c.v2.y * invr);
        *rec2 = make_float4(c.v2.x, invr, c.v2.x * B, B);
        *rec3 = make_float4(-(float)(ip.alpha * ip.h) * fabsf(c.v2.w), c.v2.w, __int_as_float(j), 0.f);
    }
    // one (target, record) pair; `valid` is false for idle lanes; kCls: the
    // class of every target (kAnyTargets: read per target)
    template <bool kStats, int kCls = kAnyTargets>
    __device__ static void pair(const InteractArgs &a, const Inst &ip, const T &t, int ti, bool valid,
                                const float4 &r0, const float4 &r1, const float4 &r2,
                                const float4 &r3, Acc<float> &acc, Counters &cn, Stats &st) {
        const float csf = (float)ip.cs;
        const bool fi = kCls == kFluidTargets ? true : kCls == kBoundaryTargets ? false : t.fluid();
        const bool fj = r3.y > 0.f;
        const float sx = fmaf(r0.y - t.a.w, csf, r0.x);
        const float dx = sx - t.a.x;
        const float dy = r0.z - t.a.y;
        const float dz = r0.w - t.a.z;
        const float rr = sq_sum_f32(dx, dy, dz);
        const int j = __float_as_int(r3.z);
        // boundary-boundary pairs are never staged, so the support decides.
        // The pair with itself (r = 0) adds zero to every sum but the delta
        // term, where the fused difference leaves the rounding error of
        // (rho_i - rho0) B_i (a relative 2^-24 of it, far inside the
        // tolerance); it is left out only where neighbours are counted per
        // particle
        const bool in = kStats ? valid && rr < (float)ip.r2max && j != ti
                               : valid && rr < (float)ip.r2max;
        cn.in += in ? 1u : 0u;
        if (kStats && in) {
            if (fj)
                ++st.f;
            else
                ++st.b;
            st.h += id_hash(a.id[j] & 0x7fffffffu);
        }
        // evaluated on every lane (no branch); lanes outside the support
        // are zeroed through F and the |mu| select
        const float r = __builtin_amdgcn_sqrtf(rr);
        // 1 - q/2 clamped to [0, 1] (the clamp is an output modifier of the
        // FMA): F vanishes outside the support without a select.  The clamp
        // and the predicate can disagree only where F is within rounding of
        // zero; counts and |mu| keep the exact predicate, and where
        // neighbours are counted per particle (kStats) F follows it too.
        // Idle lanes (valid false: kernels without sentinel records) are
        // zeroed by a select, which folds away where valid is always true.
        const float q2 =
            __builtin_amdgcn_fmed3f(fmaf(r, -0.5f * (float)ip.invh, 1.f), 0.f, 1.f);
        const float Fr = q2 * q2 * q2;  // (1-q/2)^3; store() applies m 5 w_D/h^2
        const float F = kStats ? (in ? Fr : 0.f) : (valid ? Fr : 0.f);
        const float vx = r1.x - t.b.x, vy = r1.y - t.b.y, vz = r1.z - t.b.z;
        const float vr = vx * dx + vy * dy + vz * dz;               // u_ij . r_ij
        if constexpr (kCls == kBoundaryTargets) {
            // continuity over fluid j, and |mu| for the time step; nothing else
            const float mu = vr * __builtin_amdgcn_rcpf(rr + (float)ip.eta2);  // mu / h
            acc.mu = max_abs(acc.mu, in ? mu : 0.f);
            acc.dr -= F * vr;
            return;
        }
        // one reciprocal for mu / h = vr / (r^2 + eta^2) and the viscosity's
        // mu / (h (rho_i + rho_j)) = hvi; the factor h is in the -alpha |c|
        // terms of target and record, and store() applies it to max |mu|
        const float rsum = t.c.w + r2.x;  // rho_i + rho_j (t.c.w: the target's part)
        const float hvi = vr * __builtin_amdgcn_rcpf((rr + (float)ip.eta2) * rsum);
        const float mu = hvi * rsum;
        acc.mu = max_abs(acc.mu, in ? mu : 0.f);
        acc.dr -= F * vr;                                    // m (u_i - u_j) . grad_i W_ij
        const float Fd = kCls == kFluidTargets ? F : fi ? F : 0.f;
        acc.dr += fmaf(-t.c.y, r2.w, r2.z) * Fd;             // delta term
        const float visc = (t.c.z + r3.x) * fminf(hvi, 0.f);  // -alpha h (c_i + c_j) hvi if vr < 0
        const float s = (fmaf(t.b.w, r2.y, r1.w) * t.c.x + visc) * Fd;
        acc.ax -= s * dx;
        acc.ay -= s * dy;
        acc.az -= s * dz;
    }
    // Two-phase form of pair(): the neighbour test alone, then the terms of
    // a known neighbour.  disp() is the displacement and r^2 in the
    // predicate's operation order.
    __device__ static float disp(const Inst &ip, const T &t, const float4 &r0, float &dx, float &dy,
                                 float &dz) {
        const float sx = fmaf(r0.y - t.a.w, (float)ip.cs, r0.x);
        dx = sx - t.a.x;
        dy = r0.z - t.a.y;
        dz = r0.w - t.a.z;
        return sq_sum_f32(dx, dy, dz);
    }
    __device__ static bool filter(const Inst &ip, const T &t, int ti, const float4 &r0,
                                  const float4 &r3, bool &fj) {
        fj = r3.y > 0.f;
        float dx, dy, dz;
        const float rr = disp(ip, t, r0, dx, dy, dz);
        return rr < (float)ip.r2max && __float_as_int(r3.z) != ti && (t.fluid() || fj);
    }
    template <bool kStats>
    __device__ static void body(const InteractArgs &a, const Inst &ip, const T &t, bool valid,
                                const float4 &r0, const float4 &r1, const float4 &r2,
                                const float4 &r3, Acc<float> &acc, Stats &st) {
        const bool fi = t.fluid();
        float dx, dy, dz;
        const float rr = disp(ip, t, r0, dx, dy, dz);
        if (kStats && valid) {
            if (r3.y > 0.f)
                ++st.f;
            else
                ++st.b;
            st.h += id_hash(a.id[__float_as_int(r3.z)] & 0x7fffffffu);
        }
        const float r = __builtin_amdgcn_sqrtf(rr);
        const float q2 = fmaf(r, -0.5f * (float)ip.invh, 1.f);
        const float F = valid ? q2 * q2 * q2 : 0.f;
        const float vx = r1.x - t.b.x, vy = r1.y - t.b.y, vz = r1.z - t.b.z;
        const float vr = vx * dx + vy * dy + vz * dz;
        const float rsum = t.c.w + r2.x;  // rho_i + rho_j (t.c.w: the target's part)
        const float hvi = vr * __builtin_amdgcn_rcpf((rr + (float)ip.eta2) * rsum);
        const float mu = hvi * rsum;
        acc.mu = valid ? max_nonneg(acc.mu, fabsf(mu)) : acc.mu;
        acc.dr -= F * vr;
        const float Fd = fi ? F : 0.f;
        acc.dr += fmaf(-t.c.y, r2.w, r2.z) * Fd;
        const float visc = (t.c.z + r3.x) * fminf(hvi, 0.f);  // -alpha h (c_i + c_j) hvi if vr < 0
        const float s = (fmaf(t.b.w, r2.y, r1.w) * t.c.x + visc) * Fd;
        acc.ax -= s * dx;
        acc.ay -= s * dy;
        acc.az -= s * dz;
    }
    // final sums of target i: + g for fluid; optional store of the rates;
    // the particle's time-step bound (eq. sphdt); FP64 accelerations out
    // (the sums arrive without the factors the pair terms leave out: m 5 w_D /
    // h^2 of the gradient and h of mu; they are applied here, in place)
    __device__ static void store(const InteractArgs &a, const Inst &ip, int i, bool fi, float &ax,
                                 float &ay, float &az, float &dr, float &mum, bool write,
                                 double &bound, double &oax, double &oay, double &oaz) {
        const float fm = (float)ip.Fm;
        ax *= fm;
        ay *= fm;
        az *= fm;
        dr *= fm;
        mum *= (float)ip.h;
        float fax = 0.f, fay = 0.f, faz = 0.f;
        if (fi) {
            fax = ax + (float)ip.gx;
            fay = ay + (float)ip.gy;
            faz = az + (float)ip.gz;
        }
        if (write) {
            static_cast<float *>(a.ax)[i] = fax;
            static_cast<float *>(a.ay)[i] = fay;
            static_cast<float *>(a.az)[i] = faz;
            static_cast<float *>(a.drho)[i] = dr;
            static_cast<float *>(a.mumax)[i] = mum;
        }
        oax = fax;
        oay = fay;
        oaz = faz;
        bound = ip.h / (ip.c0 + (double)mum);
        if (fi) {
            const double am = sqrt((double)fax * fax + (double)fay * fay + (double)faz * faz);
            if (am > 0.0) bound = fmin(bound, sqrt(ip.h / am));
        }
    }
};

struct Fp64 {
    using R = double;
    using V4 = double4;
    static constexpr bool kMixed = false;
    // target: {x, y, z, -}, {u, P}, {1/rho (0 for boundary), rho, -alpha |c|, -}
    struct T {
        double4 a, b, c;
        __device__ bool fluid() const { return c.x > 0.0; }
    };
    struct Cand {
        double4 v0, v1;
        double2 v2;
        bool ok;
    };
    __device__ static void target(const InteractArgs &a, const Inst &ip, int i, bool act, int rowbase, int cxa,
                                  V4 &t0, V4 &t1, V4 &t2, double &bx, double &by, double &bz,
                                  bool &fi) {
        (void)rowbase;
        (void)cxa;
        // absent target far away (+1e150 m), sentinels at -1e150 m
        double4 v0 = make_double4(1e150, 1e150, 1e150, 1), v1 = make_double4(0, 0, 0, 0);
        double2 v2 = make_double2(1, 1);
        if (act) {
            v0 = static_cast<const double4 *>(a.v0)[i];
            v1 = static_cast<const double4 *>(a.v1)[i];
            v2 = static_cast<const double2 *>(a.v2)[i];
        }
        fi = act && v2.y > 0.0;
        t0 = make_double4(v0.x, v0.y, v0.z, 0.0);
        t1 = v1;
        t2 = make_double4(fi ? v2.x : 0.0, v0.w, -(ip.alpha * ip.h) * fabs(v2.y), 0.0);
        bx = v0.x;
        by = v0.y;
        bz = v0.z;
    }
    __device__ static void load(const InteractArgs &a, const Inst &ip, int j, int je, Cand &c) {
        c.ok = j < je;
        const int jj = c.ok ? j : 0;
        c.v0 = static_cast<const double4 *>(a.v0)[jj];
        c.v1 = static_cast<const double4 *>(a.v1)[jj];
        c.v2 = static_cast<const double2 *>(a.v2)[jj];
    }
    __device__ static void cull_pos(const InteractArgs &a, const Inst &ip, const Cand &c, int nbase,
                                    int cxa, int dy, int dz, double &qx, double &qy, double &qz) {
        (void)a;
        (void)nbase;
        (void)cxa;
        (void)dy;
        (void)dz;
        qx = c.v0.x;
        qy = c.v0.y;
        qz = c.v0.z;
    }
    __device__ static void rec_pos(const InteractArgs &a, const Inst &ip, const double4 &r0, int cxa, double &qx,
                                   double &qy, double &qz) {
        (void)a;
        (void)cxa;
        qx = r0.x;
        qy = r0.y;
        qz = r0.z;
    }
    __device__ static bool cand_fluid(const Cand &c) { return c.v2.y > 0.0; }
    __device__ static bool rec_fluid(const double4 &r3) { return r3.y > 0.0; }
    __device__ static void sentinel(double4 *rec0, double4 *rec1, double4 *rec2, double4 *rec3) {
        *rec0 = make_double4(-1e150, -1e150, -1e150, -1.0);
        *rec1 = make_double4(0.0, 0.0, 0.0, 0.0);
        *rec2 = *rec1;
        *rec3 = *rec1;
    }
    // record: {x, y, z, index}, {u, P/rho}, {1/rho, B, rho, -}, {-, +-c, -, -alpha |c|}
    __device__ static void stage(const InteractArgs &a, const Inst &ip, const Cand &c, int nbase,
                                 int j, int dy, int dz, double4 *rec0, double4 *rec1, double4 *rec2,
                                 double4 *rec3) {
        (void)nbase;
        (void)dy;
        (void)dz;
        const double invr = c.v2.x;
        const bool fj = c.v2.y > 0.0;
        const double B = (fj || ip.delta_all) ? ip.kdelta * invr : 0.0;
        *rec0 = make_double4(c.v0.x, c.v0.y, c.v0.z, (double)j);
        *rec1 = make_double4(c.v1.x, c.v1.y, c.v1.z, c.v1.w * invr);
        *rec2 = make_double4(invr, B, c.v0.w, 0.0);
        *rec3 = make_double4(0.0, c.v2.y, 0.0, -(ip.alpha * ip.h) * fabs(c.v2.y));
    }
    template <bool kStats, int kCls = kAnyTargets>
    __device__ static void pair(const InteractArgs &a, const Inst &ip, const T &t, int ti, bool valid,
                                const double4 &r0, const double4 &r1, const double4 &r2,
                                const double4 &r3, Acc<double> &acc, Counters &cn, Stats &st) {
        const bool fi = kCls == kFluidTargets ? true : kCls == kBoundaryTargets ? false : t.fluid();
        const bool fj = r3.y > 0.0;
        const double dx = r0.x - t.a.x, dy = r0.y - t.a.y, dz = r0.z - t.a.z;
        const double rr = sq_sum_f64(dx, dy, dz);
        const int j = (int)r0.w;
        // as in Mixed: the support decides; the pair with itself is left out
        // only where the neighbours are counted per particle
        const bool in = kStats ? valid && rr < ip.r2max && j != ti : valid && rr < ip.r2max;
        cn.in += in ? 1u : 0u;
        if (kStats && in) {
            if (fj)
                ++st.f;
            else
                ++st.b;
            st.h += id_hash(a.id[j] & 0x7fffffffu);
        }
        // evaluated on every lane (no branch); lanes outside the support
        // are zeroed through F and the |mu| select
        const double q2 = 1.0 - 0.5 * (sqrt(rr) * ip.invh);
        const double Fr = q2 * q2 * q2;  // store() applies m 5 w_D/h^2
        const double F = in ? Fr : 0.0;
        const double vx = r1.x - t.b.x, vy = r1.y - t.b.y, vz = r1.z - t.b.z;
        const double vr = vx * dx + vy * dy + vz * dz;
        if constexpr (kCls == kBoundaryTargets) {
            // continuity over fluid j, and |mu| for the time step; nothing else
            const double mu = vr / (rr + ip.eta2);  // mu / h
            const double amu = in ? fabs(mu) : 0.0;
            acc.mu = fmax(acc.mu, amu);
            acc.dr -= F * vr;
            return;
        }
        // one division for mu = h vr / (r^2 + eta^2) and the viscosity's
        // mu / (rho_i + rho_j)
        const double rsum = t.c.y + r2.z;  // rho_i + rho_j
        const double hvi = vr / ((rr + ip.eta2) * rsum);  // h and the -alpha h |c| terms as in Mixed
        const double mu = hvi * rsum;
        const double amu = in ? fabs(mu) : 0.0;
        acc.mu = fmax(acc.mu, amu);
        acc.dr -= F * vr;
        const double Fd = kCls == kFluidTargets ? F : fi ? F : 0.0;
        acc.dr += (r2.z - t.c.y) * r2.y * Fd;
        const double visc = (t.c.z + r3.w) * fmin(hvi, 0.0);  // -alpha h (c_i + c_j) hvi if vr < 0
        const double s = (fma(t.b.w, r2.x, r1.w) * t.c.x + visc) * Fd;
        acc.ax -= s * dx;
        acc.ay -= s * dy;
        acc.az -= s * dz;
    }
    __device__ static bool filter(const Inst &ip, const T &t, int ti, const double4 &r0,
                                  const double4 &r3, bool &fj) {
        fj = r3.y > 0.0;
        const double dx = r0.x - t.a.x, dy = r0.y - t.a.y, dz = r0.z - t.a.z;
        const double rr = sq_sum_f64(dx, dy, dz);
        return rr < ip.r2max && (int)r0.w != ti && (t.fluid() || fj);
    }
    template <bool kStats>
    __device__ static void body(const InteractArgs &a, const Inst &ip, const T &t, bool valid,
                                const double4 &r0, const double4 &r1, const double4 &r2,
                                const double4 &r3, Acc<double> &acc, Stats &st) {
        const bool fi = t.fluid();
        const double dx = r0.x - t.a.x, dy = r0.y - t.a.y, dz = r0.z - t.a.z;
        const double rr = sq_sum_f64(dx, dy, dz);
        if (kStats && valid) {
            if (r3.y > 0.0)
                ++st.f;
            else
                ++st.b;
            st.h += id_hash(a.id[(int)r0.w] & 0x7fffffffu);
        }
        const double q2 = 1.0 - 0.5 * (sqrt(rr) * ip.invh);
        const double F = valid ? q2 * q2 * q2 : 0.0;
        const double vx = r1.x - t.b.x, vy = r1.y - t.b.y, vz = r1.z - t.b.z;
        const double vr = vx * dx + vy * dy + vz * dz;
        const double rsum = t.c.y + r2.z;  // rho_i + rho_j
        const double hvi = vr / ((rr + ip.eta2) * rsum);  // h and the -alpha h |c| terms as in Mixed
        const double mu = hvi * rsum;
        acc.mu = valid ? fmax(acc.mu, fabs(mu)) : acc.mu;
        acc.dr -= F * vr;
        const double Fd = fi ? F : 0.0;
        acc.dr += (r2.z - t.c.y) * r2.y * Fd;
        const double visc = (t.c.z + r3.w) * fmin(hvi, 0.0);  // -alpha h (c_i + c_j) hvi if vr < 0
        const double s = (fma(t.b.w, r2.x, r1.w) * t.c.x + visc) * Fd;
        acc.ax -= s * dx;
        acc.ay -= s * dy;
        acc.az -= s * dz;
    }
    __device__ static void store(const InteractArgs &a, const Inst &ip, int i, bool fi,
                                 double &ax, double &ay, double &az, double &dr, double &mum,
                                 bool write, double &bound, double &oax, double &oay,
                                 double &oaz) {
        ax *= ip.Fm;
        ay *= ip.Fm;
        az *= ip.Fm;
        dr *= ip.Fm;
        mum *= ip.h;
        double fax = 0, fay = 0, faz = 0;
        if (fi) {
            fax = ax + ip.gx;
            fay = ay + ip.gy;
            faz = az + ip.gz;
        }
        if (write) {
            static_cast<double *>(a.ax)[i] = fax;
            static_cast<double *>(a.ay)[i] = fay;
            static_cast<double *>(a.az)[i] = faz;
            static_cast<double *>(a.drho)[i] = dr;
            static_cast<double *>(a.mumax)[i] = mum;
        }
        oax = fax;
        oay = fay;
        oaz = faz;
        bound = ip.h / (ip.c0 + mum);
        if (fi) {
            const double am = sqrt(fax * fax + fay * fay + faz * faz);
            if (am > 0.0) bound = fmin(bound, sqrt(ip.h / am));
        }
    }
};

// The candidate ranges of a chunk of cells cxa..cxb of local half-row `lh`
// (2 row + half).  Range q in [0, 18): stencil row q / 2 (dz, dy in -1..1,
// y fastest), half q % 2 (0 fluid, 1 boundary), cells [cxa - 1, cxb + 1]
// clamped to the grid: one contiguous sorted range [js, je).  A boundary
// chunk skips the boundary halves (boundary-boundary pairs do not interact),
// so its candidates are the fluid particles near it only.  hb is the key of
// cell x = 0 of the half-row (a candidate's cell x is its key - hb); code
// packs (dy + 1) | (dz + 1) << 2.
constexpr int kRanges = 18;

// Workgroup -> work item.  The hardware deals workgroups to the XCDs in turn;
// with run > 1 the workgroups one XCD receives take runs of `run`
// consecutive items (the XCDs in turn), so neighbouring chunks, which stream
// mostly the same candidate rows, share that XCD's L2, while every XCD still
// gets a share of every part of the domain (a contiguous eighth per XCD left
// some XCDs the dry walls and others the dense water: 18 % slower).  run = 1
// is the identity.  The autotuner picks run per problem: on the 5.8 M-particle
// dam break runs of 32 cut the interaction's fetched bytes from 6.1 to
// 2.5 GB per launch and the step by ~2 %; the 64-instance ensemble gains
// ~2 % with runs of 8 (and nothing with 32).
__device__ __forceinline__ uint32_t xcd_item(uint32_t b, uint32_t run) {
    const uint32_t x = b % (uint32_t)kXcds, k = b / (uint32_t)kXcds;
    return ((k / run) * (uint32_t)kXcds + x) * run + k % run;
}
// a grid of whole XCD rounds covering `items` workgroups for xcd_item()
static uint32_t xcd_grid(uint32_t items, uint32_t run) {
    const uint32_t span = (uint32_t)kXcds * run;
    return (items + span - 1) / span * span;
}

__device__ __forceinline__ void stencil_range(const InteractArgs &a, const Inst &ip, int q, int lh,
                                              int cxa, int cxb, int &js, int &je, int &hb,
                                              int &code) {
    const int rr = q >> 1, half = q & 1;
    const int dz = rr / 3 - 1, dy = rr % 3 - 1;
    const int row = lh >> 1;
    const int czn = row / ip.ny + dz, cyn = row % ip.ny + dy;
    code = (dy + 1) | ((dz + 1) << 2);
    js = 0;
    je = 0;
    hb = 0;
    if (czn >= 0 && czn < ip.nz && cyn >= 0 && cyn < ip.ny && !((lh & 1) && half)) {
        hb = (int)half_row_key(ip, (uint32_t)(czn * ip.ny + cyn), (uint32_t)half);
        const int xlo = cxa - 1 < 0 ? 0 : cxa - 1;
        const int xhi = cxb + 1 >= ip.nx ? ip.nx - 1 : cxb + 1;
        js = (int)a.cell_start[hb + xlo];
        je = (int)a.cell_start[hb + xhi + 1];
    }
}

// The pair steps of one target group over n staged records: step s0 = 0,
// kG, 2 kG, ... < n, lane slot s taking record slot s0 + s (record index
// idx(slot), which must be valid for every slot, also past n).  body(slot,
// r0, r1, r2, r3) evaluates one step (its lanes with slot >= n are idle).
// kPipe: two register sets in alternation, the next step's records (and the
// index after it) read from LDS while this step's pair terms are evaluated;
// it costs 16 (FP32) or 32 (FP64) registers, so kernels take it only where
// their occupancy does not drop.
template <class V4, int kG, bool kPipe, class Idx, class Rec, class Body>
__device__ __forceinline__ void pair_steps(int n, int slot_s, Idx idx, Rec rec, Body body) {
    if (n <= 0) return;
    if constexpr (!kPipe) {
        for (int s0 = 0; s0 < n; s0 += kG) {
            V4 r0, r1, r2, r3;
            rec(idx(s0 + slot_s), r0, r1, r2, r3);
            body(s0 + slot_s, r0, r1, r2, r3);
        }
        return;
    }
    V4 a0, a1, a2, a3, b0, b1, b2, b3;
    int sl = slot_s;
    rec(idx(sl), a0, a1, a2, a3);
    int kb = idx(sl + kG);
    for (int s0 = 0; s0 < n; s0 += 2 * kG) {
        const bool more = s0 + kG < n;
        if (more) rec(kb, b0, b1, b2, b3);
        const int ka = idx(sl + 2 * kG);
        body(sl, a0, a1, a2, a3);
        if (!more) break;
        if (s0 + 2 * kG < n) rec(ka, a0, a1, a2, a3);
        kb = idx(sl + 3 * kG);
        body(sl + kG, b0, b1, b2, b3);
        sl += 2 * kG;
    }
}

// ================================================================ skeleton

// Fused steps that also write the next sort's keys: the kernels whose
// occupancy is fixed by their launch attributes (mixed precision, wave per
// group; row split with groups of 16 or more), so the key costs no waves.
template <class P, int kT>
constexpr bool kFusedKeys = P::kMixed && kT >= 16;

// Mixed precision with groups of 16 or more: the accumulators of the chunk's
// groups fit 128 registers, four waves per SIMD (a few spilled values
// outside the pair loop cost less than the occupancy)
template <class P, int kSplit, int kT, bool kStats, bool kFuse>
__global__ __launch_bounds__(kWave *kSplit)
__attribute__((amdgpu_waves_per_eu(P::kMixed && kT >= 16 ? 4 : 1))) void k_interact(InteractArgs a) {
    using R = typename P::R;
    using V4 = typename P::V4;
    constexpr int kRows = 2 * (9 / kSplit);  // candidate ranges per wave
    constexpr int kG = kWave / kT;  // target groups per chunk = records per step
    // mixed: record slot kWave holds a sentinel (a record outside every
    // support) and each group's list is padded with it up to a whole pair
    // step, so a step tests neither its slot nor its target
    constexpr bool kSentinel = P::kMixed;
    // staged records collect over batches and are paired once another batch
    // might not fit, so batches with few survivors share the group setup and
    // the padding of each group's list to whole pair steps: mixed precision
    // with one wave per chunk has room for 88 records (what the LDS of 16
    // blocks per CU leaves), elsewhere every batch is paired at once
    constexpr int kCap = (P::kMixed && kSplit == 1) ? 88 : kWave;
    __shared__ V4 stg[kSplit][4][kCap + 1];            // staged candidate records (per wave)
    __shared__ V4 tgt[3][kWave];                       // the chunk's targets
    __shared__ R gbox[kG][6];                          // group bounding boxes, chunk frame
    // per group: the staged records that reach it, as byte offsets into the
    // wave's staging region (a pair step adds them to a constant base)
    __shared__ uint16_t glist[kSplit][kG][kCap + kG];
    constexpr int kRecBytes = (int)sizeof(V4);
    constexpr int kRecStride = (kCap + 1) * kRecBytes;  // between the four record arrays
    __shared__ int4 rows[kSplit][kRows];
    // after its loop a wave reuses its own staging region for its per-target
    // sums (5 values of R and 3 int32 per target fit in 4 V4 per lane)
    static_assert(sizeof(R) * 5 + 4 * 3 <= sizeof(V4) * 4, "reduction fits the staging region");
    auto red = [&](int wave, int f, int idx) -> R & {
        return reinterpret_cast<R *>(&stg[wave][0][0])[f * kWave + idx];
    };
    auto redi = [&](int wave, int f, int idx) -> int32_t & {
        return reinterpret_cast<int32_t *>(reinterpret_cast<R *>(&stg[wave][0][0]) +
                                           5 * kWave)[f * kWave + idx];
    };

    const int w = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    Counters cn;
    __shared__ uint32_t wg_pairs[3];
    if (threadIdx.x < 3) wg_pairs[threadIdx.x] = 0u;  // ordered by the barrier below
    // One workgroup per chunk (in the XCD-run order of xcd_item); the grid
    // covers the most chunks the cells can produce, in whole XCD rounds, and
    // the workgroups past the current count exit at once.  The hardware
    // dispatcher balances the uneven chunk costs (dense water, dry walls)
    // with no shared counter to contend for.
    {
    const uint32_t chunk = xcd_item(blockIdx.x, a.xcd_run);
    if (chunk >= a.sc->nchunks) return;
    const int4 ch = a.chunks[chunk];
    const int cs0 = uni(ch.x), cs1 = uni(ch.y), lh = uni(ch.z), inst = uni(ch.w);
    const Inst ip = a.I.get(inst);
    const int ntgt = cs1 - cs0;
    const int rowbase = (int)half_row_key(ip, lh >> 1, lh & 1);
    const int cxa = uni((int)key_cell(a.keys[cs0]) - rowbase);
    const int cxb = uni((int)key_cell(a.keys[cs1 - 1]) - rowbase);

    // targets (lane = target index in the chunk) and their group boxes
    const int it = cs0 + lane;
    const bool act = lane < ntgt;
    R bx, by, bz;
    bool fi_own;
    {
        V4 t0, t1, t2;
        P::target(a, ip, it, act, rowbase, cxa, t0, t1, t2, bx, by, bz, fi_own);
        if (w == 0) {
            tgt[0][lane] = t0;
            tgt[1][lane] = t1;
            tgt[2][lane] = t2;
        }
    }
    const R big = (R)3.0e38f;
    {
        const R lx = group_min(act ? bx : big, kT), hx = group_max(act ? bx : -big, kT);
        const R ly = group_min(act ? by : big, kT), hy = group_max(act ? by : -big, kT);
        const R lz = group_min(act ? bz : big, kT), hz = group_max(act ? bz : -big, kT);
        if (w == 0 && lane % kT == 0) {
            const int g = lane / kT;
            gbox[g][0] = lx;
            gbox[g][1] = hx;
            gbox[g][2] = ly;
            gbox[g][3] = hy;
            gbox[g][4] = lz;
            gbox[g][5] = hz;
        }
    }
    const R lox = uni(group_min(act ? bx : big, kWave)), hix = uni(group_max(act ? bx : -big, kWave));
    const R loy = uni(group_min(act ? by : big, kWave)), hiy = uni(group_max(act ? by : -big, kWave));
    const R loz = uni(group_min(act ? bz : big, kWave)), hiz = uni(group_max(act ? bz : -big, kWave));
    const uint64_t fluid_tgts = __ballot(fi_own);
    const bool any_fluid = fluid_tgts != 0ull;
    const R cull2 = (R)(ip.r2max * (1.0 + 1e-3));

    // this wave's candidate ranges: {first, end, half-row key base, code}
    if (lane < kRows) {
        int js, je, hb, code;
        stencil_range(a, ip, w * kRows + lane, lh, cxa, cxb, js, je, hb, code);
        rows[w][lane] = make_int4(js, je, hb, code);
    }
    if constexpr (kSentinel) {
        if (lane == 0) P::sentinel(&stg[w][0][kCap], &stg[w][1][kCap], &stg[w][2][kCap],
                                   &stg[w][3][kCap]);
    }
    __syncthreads();  // targets, group boxes, rows (and the sentinel) are in LDS

    auto next_row = [&](int q) {
        while (q < kRows && rows[w][q].x >= rows[w][q].y) ++q;
        return q;
    };

    // lane -> (target t of a group, record slot s)
    const int t_in_g = lane % kT;
    const int slot_s = lane / kT;
    Acc<R> acc[kG];
    Stats sts[kG];

    // Staged records not yet paired (uniform): [0, fill) of the wave's region.
    int fill = 0;
    // Pairs the staged records: per group the records that can reach the
    // group's box, then the pair steps over them.
    auto flush = [&]() __attribute__((always_inline)) {
        wave_sync();  // the staged records
        const int cnt = fill;
        fill = 0;
        if (cnt == 0) return;
        int gcnt[kG];
#pragma unroll
        for (int g = 0; g < kG; ++g) gcnt[g] = 0;
#pragma unroll
        for (int r0 = 0; r0 < kCap; r0 += kWave) {
            if (r0 >= cnt) break;  // (uniform)
            const int r = r0 + lane;
            R px = 0, py = 0, pz = 0;
            bool rf = false;
            if (r < cnt) {
                const V4 q0 = stg[w][0][r];
                const V4 q3 = stg[w][3][r];
                P::rec_pos(a, ip, q0, cxa, px, py, pz);
                rf = P::rec_fluid(q3);
            }
#pragma unroll
            for (int g = 0; g < kG; ++g) {
                const uint64_t gbits = kT == 64 ? ~0ull : (((1ull << (kT % 64)) - 1) << (g * kT % 64));
                const bool gf = (fluid_tgts & gbits) != 0ull;
                const R ex = fmax(fmax(gbox[g][0] - px, px - gbox[g][1]), (R)0);
                const R ey = fmax(fmax(gbox[g][2] - py, py - gbox[g][3]), (R)0);
                const R ez = fmax(fmax(gbox[g][4] - pz, pz - gbox[g][5]), (R)0);
                const bool k = r < cnt && (ex * ex + ey * ey + ez * ez) <= cull2 && (gf || rf);
                const uint64_t gm = __ballot(k);
                if (k) glist[w][g][gcnt[g] + rank_below(gm)] = (uint16_t)(r * kRecBytes);
                gcnt[g] = uni(gcnt[g] + (int)__popcll(gm));
            }
        }
        if constexpr (kSentinel) {
#pragma unroll
            for (int g = 0; g < kG; ++g)
                if (lane < kG) glist[w][g][gcnt[g] + lane] = (uint16_t)(kCap * kRecBytes);
        }
        wave_sync();
#pragma unroll
        for (int g = 0; g < kG; ++g) {
            if (gcnt[g] == 0) continue;
            const int tidx = g * kT + t_in_g;
            typename P::T tg;
            tg.a = tgt[0][tidx];
            tg.b = tgt[1][tidx];
            tg.c = tgt[2][tidx];
            const int ti = cs0 + tidx;
            const int gn = gcnt[g];
            auto steps = [&](auto cls) __attribute__((always_inline)) {
                pair_steps<V4, kG, false>(
                    gn, slot_s,
                    [&](int sl) { return kSentinel || sl < gn ? (int)glist[w][g][sl] : 0; },
                    [&](int off, V4 &r0, V4 &r1, V4 &r2, V4 &r3) {
                        const char *rb = reinterpret_cast<const char *>(&stg[w][0][0]) + off;
                        r0 = *reinterpret_cast<const V4 *>(rb);
                        r1 = *reinterpret_cast<const V4 *>(rb + kRecStride);
                        r2 = *reinterpret_cast<const V4 *>(rb + 2 * kRecStride);
                        r3 = *reinterpret_cast<const V4 *>(rb + 3 * kRecStride);
                    },
                    [&](int sl, const V4 &r0, const V4 &r1, const V4 &r2, const V4 &r3) {
                        P::template pair<kStats, decltype(cls)::value>(
                            a, ip, tg, ti, kSentinel || (sl < gn && tidx < ntgt), r0, r1, r2,
                            r3, acc[g], cn, sts[g]);
                    });
            };
            // a pair body per target class (the chunk is all fluid or all
            // boundary) where the occupancy is fixed by the launch
            // attributes; elsewhere one body for both (two would cost this
            // kernel's occupancy)
            if constexpr (P::kMixed && kT >= 16) {
                if (any_fluid)
                    steps(std::integral_constant<int, kFluidTargets>{});
                else
                    steps(std::integral_constant<int, kBoundaryTargets>{});
            } else {
                steps(std::integral_constant<int, kAnyTargets>{});
            }
        }
        wave_sync();  // before the next records are staged over these
    };
    // One batch of 64 candidates (row q, first index jb): cull against the
    // chunk box and append the survivors to the staged records; pair them
    // when another batch might not fit.
    auto process = [&](const typename P::Cand &cur, int q, int jb) __attribute__((always_inline)) {
        const int4 rq = rows[w][q];
        const int dy = (rq.w & 3) - 1, dz = (rq.w >> 2) - 1;
        bool keep = false;
        if (cur.ok) {
            R qx, qy, qz;
            P::cull_pos(a, ip, cur, rq.z, cxa, dy, dz, qx, qy, qz);
            const R ex = fmax(fmax(lox - qx, qx - hix), (R)0);
            const R ey = fmax(fmax(loy - qy, qy - hiy), (R)0);
            const R ez = fmax(fmax(loz - qz, qz - hiz), (R)0);
            keep = (ex * ex + ey * ey + ez * ez) <= cull2 && (any_fluid || P::cand_fluid(cur));
        }
        const uint64_t m = __ballot(keep);
        if (keep) {
            const int slot = fill + rank_below(m);  // < kCap: fill <= kCap - kWave here
            P::stage(a, ip, cur, rq.z, jb + lane, dy, dz, &stg[w][0][slot], &stg[w][1][slot],
                     &stg[w][2][slot], &stg[w][3][slot]);
        }
        fill = uni(fill + (int)__popcll(m));
        if (fill > kCap - kWave) flush();
    };
    // the batch after (q, jb): the next 64 of the row, else the next non-empty row
    auto next_batch = [&](int q, int jb, int &q2, int &jb2) __attribute__((always_inline)) {
        q2 = q;
        jb2 = jb + kWave;
        if (jb2 >= rows[w][q].y) {
            q2 = uni(next_row(q + 1));
            jb2 = q2 < kRows ? uni(rows[w][q2].x) : 0;
        }
    };
    // (a batch past the last row loads nothing useful: every lane not ok)
    auto load_batch = [&](int q, int jb, typename P::Cand &c) __attribute__((always_inline)) {
        const bool has = q < kRows;
        const int je = has ? rows[w][has ? q : 0].y : 0;
        P::load(a, ip, has ? jb + lane : 0, je, c);
    };
    // two candidate register sets in alternation: the loads of the next
    // batch are in flight while the current one is processed
    typename P::Cand ca, cb;
    int qa = uni(next_row(0));
    int ja = qa < kRows ? uni(rows[w][qa].x) : 0;
    load_batch(qa, ja, ca);
    while (qa < kRows) {
        int qb, jbb;
        next_batch(qa, ja, qb, jbb);
        load_batch(qb, jbb, cb);
        process(ca, qa, ja);
        if (qb >= kRows) break;
        next_batch(qb, jbb, qa, ja);
        load_batch(qa, ja, ca);
        process(cb, qb, jbb);
    }
    flush();

    // sum the kG lanes that share a target (fixed shuffle tree); each wave's
    // per-target sums go to LDS
#pragma unroll
    for (int g = 0; g < kG; ++g) {
        for (int off = kT; off < kWave; off <<= 1) {
            acc[g].ax += __shfl_xor(acc[g].ax, off, kWave);
            acc[g].ay += __shfl_xor(acc[g].ay, off, kWave);
            acc[g].az += __shfl_xor(acc[g].az, off, kWave);
            acc[g].dr += __shfl_xor(acc[g].dr, off, kWave);
            const R om = __shfl_xor(acc[g].mu, off, kWave);
            acc[g].mu = om > acc[g].mu ? om : acc[g].mu;
            if constexpr (kStats) {
                sts[g].f += __shfl_xor(sts[g].f, off, kWave);
                sts[g].b += __shfl_xor(sts[g].b, off, kWave);
                sts[g].h += (uint32_t)__shfl_xor((int)sts[g].h, off, kWave);
            }
        }
        if (slot_s == 0) {
            const int tidx = g * kT + t_in_g;
            red(w, 0, tidx) = acc[g].ax;
            red(w, 1, tidx) = acc[g].ay;
            red(w, 2, tidx) = acc[g].az;
            red(w, 3, tidx) = acc[g].dr;
            red(w, 4, tidx) = acc[g].mu;
            if constexpr (kStats) {
                redi(w, 0, tidx) = sts[g].f;
                redi(w, 1, tidx) = sts[g].b;
                redi(w, 2, tidx) = (int32_t)sts[g].h;
            }
        }
    }
    // the waves' pair counts (integer, order-free) for the chunk's record
    {
        const uint32_t tot = cn.total();
        if (lane == 0) atomicAdd(&wg_pairs[any_fluid ? 0 : 2], tot);
    }
    __syncthreads();
    if (w == 0) {
    // fixed summation order over the waves; lane = target index again
    R sx = red(0, 0, lane), sy = red(0, 1, lane), sz = red(0, 2, lane);
    R sd = red(0, 3, lane), sm = red(0, 4, lane);
    int32_t nf = 0, nbd = 0;
    uint32_t hs = 0;
    if constexpr (kStats) {
        nf = redi(0, 0, lane);
        nbd = redi(0, 1, lane);
        hs = (uint32_t)redi(0, 2, lane);
    }
    for (int k = 1; k < kSplit; ++k) {
        sx += red(k, 0, lane);
        sy += red(k, 1, lane);
        sz += red(k, 2, lane);
        sd += red(k, 3, lane);
        sm = red(k, 4, lane) > sm ? red(k, 4, lane) : sm;
        if constexpr (kStats) {
            nf += redi(k, 0, lane);
            nbd += redi(k, 1, lane);
            hs += (uint32_t)redi(k, 2, lane);
        }
    }
    double bound = __longlong_as_double(0x7ff0000000000000ll);
    uint32_t nkey = 0;
    if (act) {
        double fax, fay, faz;
        P::store(a, ip, it, fi_own, sx, sy, sz, sd, sm, !kFuse, bound, fax, fay, faz);
        if constexpr (kStats) {
            a.st_nf[it] = nf;
            a.st_nb[it] = nbd;
            a.st_hash[it] = hs;
        }
        if constexpr (kFuse) {
            // every chunk reads the view, a separate copy of the state, so a
            // target can be advanced as soon as its own sums are complete; dt
            // was fixed before the launch (the lagged bound or the caller's)
            const double dt = a.ist[inst].dt_last;
            const bool euler =
                a.step == 0 || (ip.verlet_ns > 0 && a.step % ip.verlet_ns == 0);
            nkey = wcsph::advance<P::kMixed, kFusedKeys<P, kT>>(a.state, ip, it, dt, euler, fax,
                                                                fay, faz, (double)sd);
        }
    }
    if constexpr (kFuse && kFusedKeys<P, kT>) {
        if (a.hist) count_next_digit(a, act, it, nkey);
    }
    bound = group_min(bound, kWave);
    // each fluid target met itself once (in the stencil row of its own cell)
    const uint32_t self = (any_fluid && !kStats) ? (uint32_t)ntgt : 0u;
    if (lane == 0)
        a.cout[chunk] = ChunkOut{bound, {wg_pairs[0] - self, 0u, wg_pairs[2]}, 0u};
    }  // w == 0
    }  // chunk
}

// ======================================================= wave-per-group
//
// Second decomposition: a work item is a group of up to kT consecutive sorted
// particles of one cell row, owned by one wave that streams the item's own
// candidates (the nine stencil rows over [cx_first - 1, cx_last + 1]) and
// culls them against the group's box directly.  Waves never wait for each
// other (no workgroup barriers, no cross-wave sums) and hold one set of
// accumulators, so they need far fewer registers than the chunk kernel and
// more of them fit on a SIMD.  Lane (t, s) works on target t and on every
// (64 / kT)-th staged record; the per-target sums are combined by the same
// fixed shuffle tree, so results are deterministic.

constexpr int kWavesPerGroupWG = 4;  // independent waves per workgroup

template <class P, int kT, bool kStats, bool kFuse>
__global__ __launch_bounds__(kWave *kWavesPerGroupWG)
__attribute__((amdgpu_waves_per_eu(P::kMixed ? 4 : 3))) void k_interact_g(InteractArgs a) {
    using R = typename P::R;
    using V4 = typename P::V4;
    constexpr int kG = kWave / kT;
    static_assert(kT == 8 || kT == 16 || kT == 64, "group size");
    // staged records per wave: the mixed form keeps up to two batches, and
    // evaluates pairs once more than one batch's worth has gathered (fewer
    // part-filled pair steps); the FP64 records are twice as large and stay
    // at one batch (more LDS would cost occupancy)
    constexpr int kCap = P::kMixed ? 2 * kWave : kWave;
    // mixed: up to kG sentinel records after the staged ones, so the last
    // pair step of a flush reads them instead of testing its slot index (the
    // FP64 form keeps the slot test: its registers are at their limit)
    constexpr bool kSentinel = P::kMixed;
    constexpr int kSlots = kCap + (kSentinel ? kG : 0);
    __shared__ V4 stg_all[kWavesPerGroupWG][4][kSlots];
    const int w = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    V4(*stg)[kSlots] = stg_all[w];
    const int t_in = lane % kT;
    const int slot_s = lane / kT;
    Counters cn;
    {
        const uint32_t item = xcd_item(blockIdx.x, a.xcd_run) * kWavesPerGroupWG + w;
        if (item >= a.sc->nchunks) return;  // waves of a workgroup are independent
        const int4 ch = a.chunks[item];
        const int cs0 = uni(ch.x), cs1 = uni(ch.y), lh = uni(ch.z), inst = uni(ch.w);
        const Inst ip = a.I.get(inst);
        const int ntgt = cs1 - cs0;
        const int rowbase = (int)half_row_key(ip, lh >> 1, lh & 1);
        const int cxa = uni((int)key_cell(a.keys[cs0]) - rowbase);
        const int cxb = uni((int)key_cell(a.keys[cs1 - 1]) - rowbase);

        // the target of this lane (every slot lane of target t loads it)
        const int it = cs0 + t_in;
        const bool act = t_in < ntgt;
        typename P::T tg;
        R bx, by, bz;
        bool fi_own;
        P::target(a, ip, it, act, rowbase, cxa, tg.a, tg.b, tg.c, bx, by, bz, fi_own);
        const R big = (R)3.0e38f;
        // the group's box, uniform over the wave (scalar registers)
        const R lox = uni(group_min(act ? bx : big, kWave)), hix = uni(group_max(act ? bx : -big, kWave));
        const R loy = uni(group_min(act ? by : big, kWave)), hiy = uni(group_max(act ? by : -big, kWave));
        const R loz = uni(group_min(act ? bz : big, kWave)), hiz = uni(group_max(act ? bz : -big, kWave));
        const bool any_fluid = __ballot(fi_own) != 0ull;
        const R cull2 = (R)(ip.r2max * (1.0 + 1e-3));

        // candidate ranges: lane q < kRanges holds range q's {first, end,
        // half-row key base, dy/dz code}
        int r_js = 0, r_je = 0, r_nb = 0, r_code = 0;
        if (lane < kRanges) stencil_range(a, ip, lane, lh, cxa, cxb, r_js, r_je, r_nb, r_code);
        auto row_js = [&](int q) { return __builtin_amdgcn_readlane(r_js, q); };
        auto row_je = [&](int q) { return __builtin_amdgcn_readlane(r_je, q); };
        auto next_row = [&](int q) {
            while (q < kRanges && row_js(q) >= row_je(q)) ++q;
            return q;
        };
        auto next_batch = [&](int q, int jb, int &q2, int &jb2) __attribute__((always_inline)) {
            q2 = q;
            jb2 = jb + kWave;
            if (jb2 >= row_je(q)) {
                q2 = next_row(q + 1);
                jb2 = q2 < kRanges ? row_js(q2) : 0;
            }
        };
        auto load_batch = [&](int q, int jb, typename P::Cand &c) __attribute__((always_inline)) {
            const bool has = q < kRanges;
            P::load(a, ip, has ? jb + lane : 0, has ? row_je(q) : 0, c);
        };

        Acc<R> acc;
        Stats sts;
        int nst = 0;  // records staged and not yet evaluated
        // the pairs of the staged records (slots [0, nst)), then an empty stage
        auto flush = [&]() __attribute__((always_inline)) {
            const int cnt = nst;
            if constexpr (kSentinel) {
                if (lane < kG)
                    P::sentinel(&stg[0][cnt + lane], &stg[1][cnt + lane], &stg[2][cnt + lane],
                                &stg[3][cnt + lane]);
            }
            wave_sync();
            // with sentinels every slot of a step is a staged record or a
            // sentinel, and an absent target lies far away: no slot or
            // target test per pair
            auto steps = [&](auto cls) __attribute__((always_inline)) {
                pair_steps<V4, kG, P::kMixed>(
                    cnt, slot_s, [&](int sl) { return kSentinel || sl < cnt ? sl : 0; },
                    [&](int k, V4 &r0, V4 &r1, V4 &r2, V4 &r3) {
                        r0 = stg[0][k];
                        r1 = stg[1][k];
                        r2 = stg[2][k];
                        r3 = stg[3][k];
                    },
                    [&](int sl, const V4 &r0, const V4 &r1, const V4 &r2, const V4 &r3) {
                        P::template pair<kStats, decltype(cls)::value>(
                            a, ip, tg, it, kSentinel || (sl < cnt && act), r0, r1, r2, r3, acc,
                            cn, sts);
                    });
            };
            if (any_fluid)
                steps(std::integral_constant<int, kFluidTargets>{});
            else
                steps(std::integral_constant<int, kBoundaryTargets>{});
            wave_sync();
            nst = 0;
        };
        auto process = [&](const typename P::Cand &cur, int q, int jb) __attribute__((always_inline)) {
            const int code = __builtin_amdgcn_readlane(r_code, q);
            const int nbase = __builtin_amdgcn_readlane(r_nb, q);
            const int dy = (code & 3) - 1, dz = (code >> 2) - 1;
            bool keep = false;
            if (cur.ok) {
                R qx, qy, qz;
                P::cull_pos(a, ip, cur, nbase, cxa, dy, dz, qx, qy, qz);
                const R ex = fmax(fmax(lox - qx, qx - hix), (R)0);
                const R ey = fmax(fmax(loy - qy, qy - hiy), (R)0);
                const R ez = fmax(fmax(loz - qz, qz - hiz), (R)0);
                keep = (ex * ex + ey * ey + ez * ez) <= cull2 && (any_fluid || P::cand_fluid(cur));
            }
            const uint64_t m = __ballot(keep);
            if (keep) {
                const int slot = nst + rank_below(m);
                P::stage(a, ip, cur, nbase, jb + lane, dy, dz, &stg[0][slot], &stg[1][slot],
                         &stg[2][slot], &stg[3][slot]);
            }
            nst += __popcll(m);
            if (nst > kCap - kWave) flush();  // the next batch might not fit
        };

        // two candidate register sets in alternation (see the chunk kernel)
        typename P::Cand ca, cb;
        int qa = next_row(0);
        int ja = qa < kRanges ? row_js(qa) : 0;
        load_batch(qa, ja, ca);
        while (qa < kRanges) {
            int qb, jbb;
            next_batch(qa, ja, qb, jbb);
            load_batch(qb, jbb, cb);
            process(ca, qa, ja);
            if (qb >= kRanges) break;
            next_batch(qb, jbb, qa, ja);
            load_batch(qa, ja, ca);
            process(cb, qb, jbb);
        }
        if (nst > 0) flush();

        // sum the slot lanes of each target (fixed shuffle tree)
        for (int off = kT; off < kWave; off <<= 1) {
            acc.ax += __shfl_xor(acc.ax, off, kWave);
            acc.ay += __shfl_xor(acc.ay, off, kWave);
            acc.az += __shfl_xor(acc.az, off, kWave);
            acc.dr += __shfl_xor(acc.dr, off, kWave);
            const R om = __shfl_xor(acc.mu, off, kWave);
            acc.mu = om > acc.mu ? om : acc.mu;
            if constexpr (kStats) {
                sts.f += __shfl_xor(sts.f, off, kWave);
                sts.b += __shfl_xor(sts.b, off, kWave);
                sts.h += (uint32_t)__shfl_xor((int)sts.h, off, kWave);
            }
        }
        double bound = __longlong_as_double(0x7ff0000000000000ll);
        if (act && slot_s == 0) {
            double fax, fay, faz;
            P::store(a, ip, it, fi_own, acc.ax, acc.ay, acc.az, acc.dr, acc.mu, !kFuse, bound,
                     fax, fay, faz);
            if constexpr (kStats) {
                a.st_nf[it] = sts.f;
                a.st_nb[it] = sts.b;
                a.st_hash[it] = sts.h;
            }
            if constexpr (kFuse) {
                const double dt = a.ist[inst].dt_last;
                const bool euler =
                    a.step == 0 || (ip.verlet_ns > 0 && a.step % ip.verlet_ns == 0);
                wcsph::advance<P::kMixed, P::kMixed>(a.state, ip, it, dt, euler, fax, fay, faz, (double)acc.dr);
            }
        }
        bound = group_min(bound, kWave);
        const uint32_t tot = cn.total();
        // each fluid target met itself once
        const uint32_t self = (any_fluid && !kStats) ? (uint32_t)ntgt : 0u;
        if (lane == 0)
            a.cout[item] = ChunkOut{bound, {any_fluid ? tot - self : 0u, 0u, any_fluid ? 0u : tot},
                                    0u};
    }
}

// ======================================================= cooperative groups
//
// Third decomposition: a chunk of kCW groups of kT targets (one cell row) per
// workgroup of kCW waves.  The waves load the chunk's candidates together,
// kCW x 64 per batch (each wave 64), cull them against the chunk's box and
// compact them into a shared pool in LDS (double buffered: one barrier per
// batch).  Each wave then culls the pool against its own group's box and
// evaluates its pairs as in the group-per-wave kernel.  The candidate stream
// is read once per chunk instead of once per group, and each wave still
// holds one set of accumulators.

constexpr int kCW = 4;  // waves (groups) per cooperative chunk

// kTwo: the pairs of a batch in two phases -- first the neighbour test of
// every (target, record) pair, appending each target's neighbours to its own
// list, then the pair terms over the lists (lane (t, s): every kG-th entry of
// target t's list), so that the costly terms run on neighbours only.  The
// lists need LDS, so this form uses one pool buffer and two barriers per
// batch.
template <class P, int kT, bool kStats, bool kFuse, bool kTwo>
__global__ __launch_bounds__(kWave *kCW) void k_interact_c(InteractArgs a) {
    using R = typename P::R;
    using V4 = typename P::V4;
    constexpr int kG = kWave / kT;
    constexpr int kBufs = kTwo ? 1 : 2;
    static_assert(kT == 8 || kT == 16, "group size");
    __shared__ V4 pool[kBufs][4][kCW * kWave];  // staged records
    __shared__ int pcnt[kBufs][kCW];            // records each wave staged per buffer
    __shared__ uint8_t tlist[kTwo ? kCW : 1][kTwo ? kT : 1][kCW * kWave];  // per target
    __shared__ R gbox[kCW][6];                 // the groups' boxes
    __shared__ uint8_t glist[kCW][kCW * kWave];  // per wave: pool records reaching its group
    __shared__ int anyf;
    const int w = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const uint32_t chunk = xcd_item(blockIdx.x, a.xcd_run);
    if (chunk >= a.sc->nchunks) return;
    const int4 ch = a.chunks[chunk];
    const int cs0 = uni(ch.x), cs1 = uni(ch.y), lh = uni(ch.z), inst = uni(ch.w);
    const Inst ip = a.I.get(inst);
    const int rowbase = (int)half_row_key(ip, lh >> 1, lh & 1);
    const int cxa = uni((int)key_cell(a.keys[cs0]) - rowbase);
    const int cxb = uni((int)key_cell(a.keys[cs1 - 1]) - rowbase);
    const int g0 = cs0 + w * kT;                    // this wave's first target
    const int ntgt = uni(cs1 - g0 < 0 ? 0 : (cs1 - g0 > kT ? kT : cs1 - g0));
    const int t_in = lane % kT;
    const int slot_s = lane / kT;
    const int it = g0 + t_in;
    const bool act = t_in < ntgt;

    typename P::T tg;
    R bx, by, bz;
    bool fi_own;
    P::target(a, ip, it, act, rowbase, cxa, tg.a, tg.b, tg.c, bx, by, bz, fi_own);
    const R big = (R)3.0e38f;
    {
        const R lx = group_min(act ? bx : big, kWave), hx = group_max(act ? bx : -big, kWave);
        const R ly = group_min(act ? by : big, kWave), hy = group_max(act ? by : -big, kWave);
        const R lz = group_min(act ? bz : big, kWave), hz = group_max(act ? bz : -big, kWave);
        if (lane == 0) {
            gbox[w][0] = lx;
            gbox[w][1] = hx;
            gbox[w][2] = ly;
            gbox[w][3] = hy;
            gbox[w][4] = lz;
            gbox[w][5] = hz;
        }
    }
    if (threadIdx.x == 0) anyf = 0;
    __syncthreads();
    const bool my_fluid = __ballot(fi_own) != 0ull;  // (every lane takes part)
    if (lane == 0 && my_fluid) atomicOr(&anyf, 1);
    // lanes that work on the same target as this one: t_in + m kT
    const uint64_t same_t = (kT == 16 ? 0x0001000100010001ull : 0x0101010101010101ull) << t_in;
    // my group's box (pair culling) and the chunk's box (shared culling)
    const R mlx = gbox[w][0], mhx = gbox[w][1], mly = gbox[w][2], mhy = gbox[w][3];
    const R mlz = gbox[w][4], mhz = gbox[w][5];
    R clx = big, chx = -big, cly = big, chy = -big, clz = big, chz = -big;
#pragma unroll
    for (int k = 0; k < kCW; ++k) {
        clx = fmin(clx, gbox[k][0]);
        chx = fmax(chx, gbox[k][1]);
        cly = fmin(cly, gbox[k][2]);
        chy = fmax(chy, gbox[k][3]);
        clz = fmin(clz, gbox[k][4]);
        chz = fmax(chz, gbox[k][5]);
    }
    const R cull2 = (R)(ip.r2max * (1.0 + 1e-3));

    // candidate ranges: lane q < kRanges holds range q's {first, end,
    // half-row key base, dy/dz code}
    int r_js = 0, r_je = 0, r_nb = 0, r_code = 0;
    if (lane < kRanges) stencil_range(a, ip, lane, lh, cxa, cxb, r_js, r_je, r_nb, r_code);
    __syncthreads();  // anyf is final
    const bool any_fluid = anyf != 0;
    auto row_js = [&](int q) { return __builtin_amdgcn_readlane(r_js, q); };
    auto row_je = [&](int q) { return __builtin_amdgcn_readlane(r_je, q); };
    auto next_row = [&](int q) {
        while (q < kRanges && row_js(q) >= row_je(q)) ++q;
        return q;
    };
    constexpr int kB = kCW * kWave;  // candidates per shared batch
    auto next_batch = [&](int q, int jb, int &q2, int &jb2) __attribute__((always_inline)) {
        q2 = q;
        jb2 = jb + kB;
        if (jb2 >= row_je(q)) {
            q2 = next_row(q + 1);
            jb2 = q2 < kRanges ? row_js(q2) : 0;
        }
    };
    auto load_batch = [&](int q, int jb, typename P::Cand &c) __attribute__((always_inline)) {
        const bool has = q < kRanges;
        P::load(a, ip, has ? jb + w * kWave + lane : 0, has ? row_je(q) : 0, c);
    };

    Acc<R> acc;
    Stats sts;
    Counters cn;
    typename P::Cand cur;
    int q = next_row(0);
    int jb = q < kRanges ? row_js(q) : 0;
    load_batch(q, jb, cur);
    int buf = 0;
    while (q < kRanges) {
        const int code = __builtin_amdgcn_readlane(r_code, q);
        const int nbase = __builtin_amdgcn_readlane(r_nb, q);
        const int dy = (code & 3) - 1, dz = (code >> 2) - 1;
        // A: cull my 64 candidates against the chunk box, stage into the pool
        bool keep = false;
        if (cur.ok) {
            R qx, qy, qz;
            P::cull_pos(a, ip, cur, nbase, cxa, dy, dz, qx, qy, qz);
            const R ex = fmax(fmax(clx - qx, qx - chx), (R)0);
            const R ey = fmax(fmax(cly - qy, qy - chy), (R)0);
            const R ez = fmax(fmax(clz - qz, qz - chz), (R)0);
            keep = (ex * ex + ey * ey + ez * ez) <= cull2 && (any_fluid || P::cand_fluid(cur));
        }
        const uint64_t m = __ballot(keep);
        if (keep) {
            const int slot = w * kWave + rank_below(m);
            P::stage(a, ip, cur, nbase, jb + w * kWave + lane, dy, dz, &pool[buf][0][slot],
                     &pool[buf][1][slot], &pool[buf][2][slot], &pool[buf][3][slot]);
        }
        if (lane == 0) pcnt[buf][w] = __popcll(m);
        // the next batch's loads are in flight during the barrier and B
        int q2, jb2;
        next_batch(q, jb, q2, jb2);
        load_batch(q2, jb2, cur);
        __syncthreads();
        // B: the pool records that reach my group, then my pairs
        if (ntgt > 0) {
            int n = 0;
#pragma unroll
            for (int k = 0; k < kCW; ++k) {
                const int cnt = pcnt[buf][k];
                bool kk = false;
                if (lane < cnt) {
                    const V4 r0 = pool[buf][0][k * kWave + lane];
                    const V4 r3 = pool[buf][3][k * kWave + lane];
                    R px, py, pz;
                    P::rec_pos(a, ip, r0, cxa, px, py, pz);
                    const R ex = fmax(fmax(mlx - px, px - mhx), (R)0);
                    const R ey = fmax(fmax(mly - py, py - mhy), (R)0);
                    const R ez = fmax(fmax(mlz - pz, pz - mhz), (R)0);
                    kk = (ex * ex + ey * ey + ez * ez) <= cull2 && (my_fluid || P::rec_fluid(r3));
                }
                const uint64_t gm = __ballot(kk);
                if (kk) glist[w][n + rank_below(gm)] = (uint8_t)(k * kWave + lane);
                n += __popcll(gm);
            }
            wave_sync();
            if constexpr (kTwo) {
                // phase 1: the neighbour test; target t's neighbours go to its list
                uint8_t *tl = tlist[w][t_in];
                int nn = 0;
                for (int s0 = 0; s0 < n; s0 += kG) {
                    const int sl = s0 + slot_s;
                    const int k = (int)glist[w][sl < n ? sl : 0];
                    const V4 r0 = pool[buf][0][k], r3 = pool[buf][3][k];
                    bool fj;
                    const bool in = P::filter(ip, tg, it, r0, r3, fj) && sl < n && act;
                    const uint64_t inm = __ballot(in);
                    cn.in += in ? 1u : 0u;
                    const uint64_t mine = inm & same_t;
                    if (in) tl[nn + rank_below(mine)] = (uint8_t)k;
                    nn += __popcll(mine);
                }
                wave_sync();
                // phase 2: the pair terms; idle lanes read a record of this
                // batch (their terms are multiplied by zero and stay finite)
                const int nmax = uni(group_max(nn, kWave));
                const int k0 = (int)glist[w][0];
                for (int s0 = 0; s0 < nmax; s0 += kG) {
                    const int sl = s0 + slot_s;
                    const bool valid = sl < nn;
                    const int k = valid ? (int)tl[sl] : k0;
                    const V4 r0 = pool[buf][0][k], r1 = pool[buf][1][k];
                    const V4 r2 = pool[buf][2][k], r3 = pool[buf][3][k];
                    P::template body<kStats>(a, ip, tg, valid, r0, r1, r2, r3, acc, sts);
                }
            } else {
                // idle lanes read a record staged in this batch (entry 0):
                // their terms are multiplied by zero and must stay finite
                auto steps = [&](auto cls) __attribute__((always_inline)) {
                    pair_steps<V4, kG, true>(
                        n, slot_s, [&](int sl) { return (int)glist[w][sl < n ? sl : 0]; },
                        [&](int k, V4 &r0, V4 &r1, V4 &r2, V4 &r3) {
                            r0 = pool[buf][0][k];
                            r1 = pool[buf][1][k];
                            r2 = pool[buf][2][k];
                            r3 = pool[buf][3][k];
                        },
                        [&](int sl, const V4 &r0, const V4 &r1, const V4 &r2, const V4 &r3) {
                            P::template pair<kStats, decltype(cls)::value>(
                                a, ip, tg, it, sl < n && act, r0, r1, r2, r3, acc, cn, sts);
                        });
                };
                if (any_fluid)
                    steps(std::integral_constant<int, kFluidTargets>{});
                else
                    steps(std::integral_constant<int, kBoundaryTargets>{});
            }
            wave_sync();
        }
        if constexpr (kTwo) __syncthreads();  // the single pool is rewritten next
        buf = (buf + 1) % kBufs;
        q = q2;
        jb = jb2;
    }

    // sum the slot lanes of each target (fixed shuffle tree)
    for (int off = kT; off < kWave; off <<= 1) {
        acc.ax += __shfl_xor(acc.ax, off, kWave);
        acc.ay += __shfl_xor(acc.ay, off, kWave);
        acc.az += __shfl_xor(acc.az, off, kWave);
        acc.dr += __shfl_xor(acc.dr, off, kWave);
        const R om = __shfl_xor(acc.mu, off, kWave);
        acc.mu = om > acc.mu ? om : acc.mu;
        if constexpr (kStats) {
            sts.f += __shfl_xor(sts.f, off, kWave);
            sts.b += __shfl_xor(sts.b, off, kWave);
            sts.h += (uint32_t)__shfl_xor((int)sts.h, off, kWave);
        }
    }
    double bound = __longlong_as_double(0x7ff0000000000000ll);
    if (act && slot_s == 0) {
        double fax, fay, faz;
        P::store(a, ip, it, fi_own, acc.ax, acc.ay, acc.az, acc.dr, acc.mu, !kFuse, bound, fax,
                 fay, faz);
        if constexpr (kStats) {
            a.st_nf[it] = sts.f;
            a.st_nb[it] = sts.b;
            a.st_hash[it] = sts.h;
        }
        if constexpr (kFuse) {
            const double dt = a.ist[inst].dt_last;
            const bool euler = a.step == 0 || (ip.verlet_ns > 0 && a.step % ip.verlet_ns == 0);
            wcsph::advance<P::kMixed, false>(a.state, ip, it, dt, euler, fax, fay, faz, (double)acc.dr);
        }
    }
    // the workgroup's bound and pair counts for the chunk's record
    __shared__ unsigned long long wb;
    __shared__ uint32_t wp[3];
    if (threadIdx.x == 0) {
        wb = 0x7ff0000000000000ull;
        wp[0] = wp[1] = wp[2] = 0u;
    }
    __syncthreads();
    bound = group_min(bound, kWave);
    const uint32_t tot = cn.total();
    // the one-phase pair body met each fluid target itself once; the
    // two-phase neighbour test leaves that pair out
    const uint32_t self = (any_fluid && !kStats && !kTwo) ? (uint32_t)ntgt : 0u;
    if (lane == 0) {
        atomicMin(&wb, (unsigned long long)__double_as_longlong(bound));
        atomicAdd(&wp[any_fluid ? 0 : 2], tot - self);
    }
    __syncthreads();
    if (threadIdx.x == 0)
        a.cout[chunk] = ChunkOut{__longlong_as_double((long long)wb), {wp[0], wp[1], wp[2]}, 0u};
}

// Per-instance minimum of the chunks' time-step bounds and the pair totals.
// Block b reduces chunks [1024 b, 1024 b + 1024): chunks are ordered by
// instance, so the block's instances are inst0 .. inst0 + 1023 at most.  A
// wave whose chunks all belong to one instance (nearly every wave) first
// reduces across its lanes by shuffles and makes one LDS update; a wave that
// straddles instances updates LDS lane by lane.  Then one global atomic per
// instance and block (a handful in all: no contention).
__global__ __launch_bounds__(1024) void k_chunk_reduce(const int4 *__restrict__ chunks,
                                                       const ChunkOut *__restrict__ cout,
                                                       DevScalars *sc, InstState *ist) {
    constexpr unsigned long long kInf = 0x7ff0000000000000ull;
    __shared__ unsigned long long smin[1024];
    __shared__ unsigned long long spairs[3];
    __shared__ int inst0;
    const uint32_t nch = sc->nchunks;
    const uint32_t c0 = blockIdx.x * 1024u;
    if (c0 >= nch) return;
    const int t = threadIdx.x;
    smin[t] = kInf;
    if (t < 3) spairs[t] = 0ull;
    if (t == 0) inst0 = chunks[c0].w;
    __syncthreads();
    const uint32_t c = c0 + (uint32_t)t;
    const bool ok = c < nch;
    unsigned long long b = kInf;
    unsigned long long p0 = 0, p1 = 0, p2 = 0;  // 64-bit: wave sums of 32-bit counts
    int slot = -1;
    if (ok) {
        const ChunkOut o = cout[c];
        b = (unsigned long long)__double_as_longlong(o.bound);
        p0 = o.pairs[0];
        p1 = o.pairs[1];
        p2 = o.pairs[2];
        slot = chunks[c].w - inst0;
    }
    const int s0 = __shfl(slot, 0, kWave);
    if (__all(slot == s0 || slot < 0)) {
        // bounds are non-negative doubles: their bit patterns order alike
        for (int off = 1; off < kWave; off <<= 1) {
            const unsigned long long ob = __shfl_xor(b, off, kWave);
            b = ob < b ? ob : b;
            p0 += __shfl_xor(p0, off, kWave);
            p1 += __shfl_xor(p1, off, kWave);
            p2 += __shfl_xor(p2, off, kWave);
        }
        if (t % kWave == 0) {
            atomicMin(&smin[s0], b);
            atomicAdd(&spairs[0], p0);
            atomicAdd(&spairs[1], p1);
            atomicAdd(&spairs[2], p2);
        }
    } else if (ok) {
        atomicMin(&smin[slot], b);
        atomicAdd(&spairs[0], p0);
        atomicAdd(&spairs[1], p1);
        atomicAdd(&spairs[2], p2);
    }
    __syncthreads();
    if (smin[t] != kInf) atomicMin(&ist[inst0 + t].dt_min_bits, smin[t]);
    if (t < 3 && spairs[t]) atomicAdd(&sc->pairs[t], spairs[t]);
}

// ================================================================ launch

// interaction launch shape per precision: waves per chunk and targets per
// group (0 = automatic).  Host-side preferences set by sph_set_tuning (the
// autotuner); atomics, so a thread that launches while another sets them
// reads defined values (each field on its own).  They pick launch shapes
// only, never results beyond summation order.
static std::atomic<int> g_split[2] = {{0}, {0}};
static std::atomic<int> g_group[2] = {{0}, {0}};
static std::atomic<int> g_kernel[2] = {{0}, {0}};
static std::atomic<int> g_xcd[2] = {{0}, {0}};

int set_xcd_run(int precision, int run) {
    if (precision != SPH_FP64 && precision != SPH_MIXED) return -1;
    if (run != 0 && run != 1 && run != 8 && run != 32) return -1;
    g_xcd[precision].store(run, std::memory_order_relaxed);
    return 0;
}

int xcd_run_for(const Problem &P) {
    const int r = g_xcd[P.precision == SPH_MIXED ? SPH_MIXED : SPH_FP64].load(
        std::memory_order_relaxed);
    return r ? r : 1;
}

// nonzero: every step gathers every particle (no fluid-only sort)
static std::atomic<int> g_full_gather{0};
void set_full_gather(int on) { g_full_gather.store(on ? 1 : 0, std::memory_order_relaxed); }
int full_gather() { return g_full_gather.load(std::memory_order_relaxed); }

int set_kernel(int precision, int kernel) {
    if (precision != SPH_FP64 && precision != SPH_MIXED) return -1;
    if (kernel != SPH_KERNEL_AUTO && kernel != SPH_KERNEL_ROWS && kernel != SPH_KERNEL_GROUPS &&
        kernel != SPH_KERNEL_COOP && kernel != SPH_KERNEL_COOP2)
        return -1;
    g_kernel[precision].store(kernel, std::memory_order_relaxed);
    return 0;
}

int kernel_for(const Problem &P) {
    const int pr = P.precision == SPH_MIXED ? SPH_MIXED : SPH_FP64;
    const int k = g_kernel[pr].load(std::memory_order_relaxed);
    return k ? k : SPH_KERNEL_ROWS;
}

bool fused_writes_keys(const Problem &P) {
    // the kernels instantiated with kFusedKeys
    if (P.precision != SPH_MIXED) return false;
    const int k = kernel_for(P);
    return k == SPH_KERNEL_GROUPS || (k == SPH_KERNEL_ROWS && group_for(P) >= 16);
}

bool fused_counts_digits(const Problem &P) {
    // the row-split kernel with kFusedKeys (one target per lane of wave 0)
    return P.precision == SPH_MIXED && kernel_for(P) == SPH_KERNEL_ROWS && group_for(P) >= 16;
}

int chunk_for(const Problem &P) {
    const int k = kernel_for(P);
    if (k == SPH_KERNEL_GROUPS) return group_for(P);
    if (k == SPH_KERNEL_COOP || k == SPH_KERNEL_COOP2) return kCW * (group_for(P) == 8 ? 8 : 16);
    return kChunk;
}

int set_split(int precision, int split) {
    if (precision != SPH_FP64 && precision != SPH_MIXED) return -1;
    if (split != 0 && split != 1 && split != 3 && split != 9) return -1;
    g_split[precision].store(split, std::memory_order_relaxed);
    return 0;
}

int set_group(int precision, int group) {
    if (precision != SPH_FP64 && precision != SPH_MIXED) return -1;
    if (group != 0 && group != 8 && group != 16 && group != 64) return -1;
    g_group[precision].store(group, std::memory_order_relaxed);
    return 0;
}

int split_for(const Problem &P) {
    const int s = g_split[P.precision == SPH_MIXED ? SPH_MIXED : SPH_FP64].load(
        std::memory_order_relaxed);
    if (s) return s;
    const int64_t max_chunks = (P.n + kChunk - 1) / kChunk + P.nrows;
    // enough waves to fill 256 CUs x 4 SIMDs several times over
    if (max_chunks < 2048) return 9;
    if (max_chunks < 16384) return 3;
    return 1;
}

int group_for(const Problem &P) {
    const int pr = P.precision == SPH_MIXED ? SPH_MIXED : SPH_FP64;
    const int g = g_group[pr].load(std::memory_order_relaxed);
    if (g) return g;
    return pr == SPH_MIXED ? 8 : 16;
}

// nb: the most chunks the cells can produce (one workgroup each)
template <class P, int kSplit, int kT, bool kStats, bool kFuse>
static void launch_one(uint32_t nb, const InteractArgs &a, hipStream_t st) {
    hipLaunchKernelGGL((k_interact<P, kSplit, kT, kStats, kFuse>), dim3(xcd_grid(nb, a.xcd_run)),
                       dim3(kWave * kSplit), 0, st, a);
}

template <class P, int kSplit, bool kStats, bool kFuse>
static void launch_group(int group, uint32_t cap, const InteractArgs &a, hipStream_t st) {
    switch (group) {
    case 8:
        launch_one<P, kSplit, 8, kStats, kFuse>(cap, a, st);
        break;
    case 16:
        launch_one<P, kSplit, 16, kStats, kFuse>(cap, a, st);
        break;
    default:
        launch_one<P, kSplit, 64, kStats, kFuse>(cap, a, st);
        break;
    }
}

template <class P, bool kStats, bool kFuse>
static void launch_shape(int split, int group, uint32_t nb, const InteractArgs &a,
                         hipStream_t st) {
    switch (split) {
    case 9:
        launch_group<P, 9, kStats, kFuse>(group, nb, a, st);
        break;
    case 3:
        launch_group<P, 3, kStats, kFuse>(group, nb, a, st);
        break;
    default:
        launch_group<P, 1, kStats, kFuse>(group, nb, a, st);
        break;
    }
}

// nb: workgroups of kWavesPerGroupWG waves covering the most chunks
template <class P, int kT, bool kStats, bool kFuse>
static void launch_g(uint32_t nb, const InteractArgs &a, hipStream_t st) {
    hipLaunchKernelGGL((k_interact_g<P, kT, kStats, kFuse>), dim3(xcd_grid(nb, a.xcd_run)),
                       dim3(kWave * kWavesPerGroupWG), 0, st, a);
}

template <class P, bool kStats, bool kFuse>
static void launch_g_group(int group, uint32_t cap, const InteractArgs &a, hipStream_t st) {
    switch (group) {
    case 8:
        launch_g<P, 8, kStats, kFuse>(cap, a, st);
        break;
    case 16:
        launch_g<P, 16, kStats, kFuse>(cap, a, st);
        break;
    default:
        launch_g<P, 64, kStats, kFuse>(cap, a, st);
        break;
    }
}

template <class P, bool kStats, bool kFuse, bool kTwo>
static void launch_c(int group, uint32_t nb, const InteractArgs &a, hipStream_t st) {
    if (group == 8)
        hipLaunchKernelGGL((k_interact_c<P, 8, kStats, kFuse, kTwo>), dim3(xcd_grid(nb, a.xcd_run)),
                           dim3(kWave * kCW), 0, st, a);
    else
        hipLaunchKernelGGL((k_interact_c<P, 16, kStats, kFuse, kTwo>), dim3(xcd_grid(nb, a.xcd_run)),
                           dim3(kWave * kCW), 0, st, a);
}

template <class P, bool kTwo>
static void launch_c_mode(int group, uint32_t nb, bool stats, bool fuse, const InteractArgs &a,
                          hipStream_t st) {
    if (stats)
        launch_c<P, true, false, kTwo>(group, nb, a, st);
    else if (fuse)
        launch_c<P, false, true, kTwo>(group, nb, a, st);
    else
        launch_c<P, false, false, kTwo>(group, nb, a, st);
}

template <class P>
static void launch_prec(int kernel, int split, int group, uint32_t nb, bool stats, bool fuse,
                        const InteractArgs &a, hipStream_t st) {
    if (kernel == SPH_KERNEL_COOP) {
        launch_c_mode<P, false>(group, nb, stats, fuse, a, st);
        return;
    }
    if (kernel == SPH_KERNEL_COOP2) {
        launch_c_mode<P, true>(group, nb, stats, fuse, a, st);
        return;
    }
    if (kernel == SPH_KERNEL_GROUPS) {
        const uint32_t cap = (nb + kWavesPerGroupWG - 1) / kWavesPerGroupWG;
        if (stats)
            launch_g_group<P, true, false>(group, cap, a, st);
        else if (fuse)
            launch_g_group<P, false, true>(group, cap, a, st);
        else
            launch_g_group<P, false, false>(group, cap, a, st);
        return;
    }
    if (stats)
        launch_shape<P, true, false>(split, group, nb, a, st);
    else if (fuse)
        launch_shape<P, false, true>(split, group, nb, a, st);
    else
        launch_shape<P, false, false>(split, group, nb, a, st);
}

int launch_interact(const Problem &P, const sph_state &s, const Ws &w, hipStream_t st,
                    int32_t *st_nf, int32_t *st_nb, uint32_t *st_hash, bool fuse,
                    int64_t step, hipEvent_t after_kernel, int count_shift) {
    InteractArgs a;
    a.xcd_run = (uint32_t)xcd_run_for(P);
    const bool count = fuse && count_shift >= 0 && st_nf == nullptr && fused_counts_digits(P);
    a.hist = count ? w.hist() : nullptr;
    a.hist_shift = count_shift;
    a.ntiles = (int)w.L.ntiles;
    a.tile_log2 = 0;
    while (((int64_t)1 << a.tile_log2) < sort_tile(s.n)) ++a.tile_log2;
    a.chunks = w.chunks();
    a.sc = w.scalars();
    a.ist = w.inst_state();
    a.I = insts_of(P, w);
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
    a.cout = w.chunk_out();
    a.id = s.id;
    a.st_nf = st_nf;
    a.st_nb = st_nb;
    a.st_hash = st_hash;
    a.state = StateArrays{s.x,   s.y,   s.z,   s.ux,   s.uy,  s.uz,
                          s.uxm, s.uym, s.uzm, s.rho,  s.rhom, s.id, w.keys_next(),
                          &w.scalars()->walls_move, s.rho_alt, s.rhom_alt};
    a.step = step;
    const bool stats = st_nf != nullptr;
    // chunks of <= csz targets: at most ceil(particles / csz) + 1 per half-row
    const int64_t csz = chunk_for(P);
    const uint32_t nb = (uint32_t)((P.n + csz - 1) / csz + 4 * P.nrows);
    const int split = split_for(P);
    const int group = group_for(P);
    const int kernel = kernel_for(P);
    if (P.precision == SPH_MIXED)
        launch_prec<Mixed>(kernel, split, group, nb, stats, fuse && !stats, a, st);
    else
        launch_prec<Fp64>(kernel, split, group, nb, stats, fuse && !stats, a, st);
    if (int rc = launch_check("interact")) return rc;
    if (after_kernel)
        if (int rc = hip_check(hipEventRecord(after_kernel, st), "event record")) return rc;
    hipLaunchKernelGGL(k_chunk_reduce, dim3((nb + 1023) / 1024), dim3(1024), 0, st, w.chunks(),
                       w.chunk_out(), w.scalars(), w.inst_state());
    return launch_check("chunk reduce");
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

int launch_export_rates(const Problem &P, const Ws &w, double *ax, double *ay, double *az,
                        double *drho, double *mumax, hipStream_t st) {
    const int64_t n = P.n;
    int blocks = (int)((n + 255) / 256);
    if (P.precision == SPH_MIXED)
        hipLaunchKernelGGL(k_export<float>, dim3(blocks), dim3(256), 0, st,
                           w.at<const float>(w.L.rates), n, ax, ay, az, drho, mumax);
    else
        hipLaunchKernelGGL(k_export<double>, dim3(blocks), dim3(256), 0, st,
                           w.at<const double>(w.L.rates), n, ax, ay, az, drho, mumax);
    return launch_check("export rates");
}

}  // namespace wcsph
