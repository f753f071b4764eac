// Internal declarations shared by the HIP translation units of libwcsph.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "wcsph.h"

namespace wcsph {

constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kSortThreads = 256;    // radix sort workgroup
constexpr int kSortItemsLarge = 16;  // keys per thread per tile (large arrays)
constexpr int kSortItemsSmall = 4;   // (up to kSortSmallN keys: more, smaller tiles)
constexpr int64_t kSortSmallN = 1 << 21;
// keys per sort tile for n keys: enough tiles to occupy the whole chip
inline int64_t sort_tile(int64_t n) {
    return (int64_t)kSortThreads * (n <= kSortSmallN ? kSortItemsSmall : kSortItemsLarge);
}
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kScanThreads = 1024;   // scan workgroup
constexpr int kScanSpan = 4 * kScanThreads;  // values per scanned span
constexpr int kScanRedundantSpans = 16;  // up to this many spans: one launch
constexpr int kScanSumSpans = 16 * kScanThreads;  // up to this many: two (totals, then spans)
constexpr int kChunk = 64;           // targets per chunk of the row-split interaction
constexpr int kMinChunk = 8;         // smallest chunk (group-per-wave interaction)
constexpr int kDiagThreads = 256;
constexpr int kDiagBlocks = 1024;    // partial sums of a single system (fixed: deterministic)
constexpr int kDiagBlocksBatch = 32; // partial sums per instance of a batch
constexpr int kDiagFields = 16;
constexpr int kMaxProbes = 1024;     // probe points per sph_diagnostics call
constexpr int64_t kMaxGraphSteps = 400;  // longest captured step sequence

// Constants of one particle system ("instance"): its grid, its slice of the
// global cell and row numbering, its particles' original ids, and the
// physical parameters.  A batch holds several; a single system is a batch of
// one.
struct Inst {
    double ox, oy, oz, cs;  // grid origin and cell edge
    double h, invh, r2max, eta2;
    double Fm;              // m * 5 w_D / h^2 (radial gradient factor times mass)
    double wd;              // kernel constant 21 / (16 pi h^3)
    double alpha, kdelta;   // kdelta = 2 delta h c0
    double rho0, c0, B, gamma;
    double gx, gy, gz;
    double cfl, mass;
    int32_t nx, ny, nz;
    int32_t c_const, delta_all, verlet_ns;
    uint32_t cell_base;     // first global cell id
    uint32_t row_base;      // first global row id (a row = fixed cy, cz)
    uint32_t pstart, pend;  // original particle ids [pstart, pend)
};

// Per-instance device state (time step and clock).
struct InstState {
    unsigned long long dt_min_bits;  // running min of this step's bound (bits of
                                     // a positive double order like integers)
    unsigned long long dt_lag_bits;  // the previous step's bound (lagged dt)
    double dt_cfl;                   // Cr * bound of the last interaction
    double dt_last;                  // dt used by the last step
    double time;                     // accumulated simulated time
    double pad;
};

// What the interaction leaves per chunk: the chunk's time-step bound
// (eq. sphdt, before the Courant factor) and its interacting pair counts:
// {FF + FB, 0, 0} for a chunk of fluid targets, {0, 0, BF} for boundary ones.
struct ChunkOut {
    double bound;
    uint32_t pairs[3];
    uint32_t pad;
};

// Running pressure impulse of the probe points (trapezoidal rule over the
// samples of sph_probe_impulse), followed in the workspace by kMaxProbes
// impulses and kMaxProbes previous pressures.
struct ImpulseState {
    double t_prev;   // simulated time of the previous sample
    int32_t has_prev;  // a previous sample exists (0 after init or reset)
    int32_t np;      // probes of the previous sample
};

// Device-wide scalars.
struct DevScalars {
    long long steps;                 // steps taken
    unsigned int nchunks;            // interaction chunks of the current cells
    unsigned int dt_cfl_violation;   // a step used dt > dt_cfl
    unsigned long long pairs[3];     // interacting pairs since init: FF + FB, 0, BF
    unsigned int walls_move;         // some step with this workspace moved a boundary
                                     // particle (nonzero velocity); never cleared
    unsigned int pad;
};

// Lanes below this one in the wave.
__device__ __forceinline__ uint64_t lanemask_lt() {
    uint32_t lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Lanes of the wave whose radix digit equals this lane's (restricted to
// `valid`): one ballot per digit bit.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t valid) {
    uint64_t peers = valid;
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        uint64_t bal = __ballot((d >> b) & 1u);
        peers &= ((d >> b) & 1u) ? bal : ~bal;
    }
    return peers;
}

// The sort tile that block b of a one-block-per-tile launch handles.  The
// hardware deals consecutive workgroups to the 8 XCDs in turn, and each XCD
// has its own L2; the blocks an XCD receives (b mod 8 equal) take a
// contiguous run of tiles, so the per-tile digit counts (digit-major,
// neighbouring tiles in one cache line) are written and read through one
// L2 instead of being written back a few bytes at a time from eight.  A
// bijection on [0, ntiles) whatever the placement.
constexpr int kXcds = 8;
__device__ __forceinline__ int tile_of_block(int b, int ntiles) {
    const int per = ntiles / kXcds, rem = ntiles % kXcds, x = b % kXcds;
    return x * per + (x < rem ? x : rem) + b / kXcds;
}

// Lanes that start a run of equal values v in consecutive lanes (lane 0
// always does).
__device__ __forceinline__ uint64_t run_starts(uint32_t v) {
    const int lane = __lane_id();
    const uint32_t prev = __shfl_up(v, 1, kWave);
    return __ballot(lane == 0 || prev != v);
}

// Length of the run that starts at this lane (starts as from run_starts).
__device__ __forceinline__ uint32_t run_length(uint64_t starts) {
    const int lane = __lane_id();
    const uint64_t later = (starts >> lane) >> 1;  // run starts above this lane
    return later ? (uint32_t)__builtin_ctzll(later) + 1u : (uint32_t)(kWave - lane);
}

// Adds a wave's keys (those with ok) to a sort tile's digit counts in LDS:
// one atomic per run of equal digits in consecutive lanes (nearly sorted
// keys come in a few long runs; a digit in several runs takes one atomic
// per run).  All lanes of the wave call it.
__device__ __forceinline__ void tile_hist_add(uint32_t *h, uint32_t key, bool ok, int shift) {
    const uint32_t d = ok ? (key >> shift) & (kRadix - 1) : (uint32_t)kRadix;  // kRadix: no key
    const uint64_t starts = run_starts(d);
    if (ok && ((starts >> __lane_id()) & 1u)) atomicAdd(&h[d], run_length(starts));
}

// Orders one wave's LDS writes before its later reads (and reads before
// later overwrites) without involving the other waves of the workgroup.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sort keys.  Every cell row (fixed cy, cz) of an instance is split into a
// fluid half-row and a boundary half-row, cells x-fastest within each.  An
// instance's keys fill [2 cell_base, 2 (cell_base + its cells)): first its
// fluid half-rows, row by row, then its boundary half-rows in the same order,
// so a run of cells of one row holds its fluid particles contiguously and its
// boundary particles contiguously, and all of an instance's boundary
// particles follow all of its fluid ones (a fixed wall's particles then keep
// their sorted positions from step to step).  The key of cell x of half-row
// `half` (0 fluid, 1 boundary) of local row `lrow` is half_row_key(...) + x.
__host__ __device__ __forceinline__ uint32_t inst_cells(const Inst &ip) {
    return (uint32_t)ip.nx * (uint32_t)ip.ny * (uint32_t)ip.nz;
}
__host__ __device__ __forceinline__ uint32_t half_row_key(const Inst &ip, uint32_t lrow,
                                                          uint32_t half) {
    return 2u * ip.cell_base + half * inst_cells(ip) + lrow * (uint32_t)ip.nx;
}
// a global cell of the cell key's row (enough to find the key's instance)
__host__ __device__ __forceinline__ uint32_t key_row_cell(uint32_t key) { return key >> 1; }

// The sort key appends kSubBits to the cell key: the half of the cell the
// particle lies in along y and along x.  Sorted on every bit, the particles
// of a cell come in four columns of half the cell's width, so runs of 8
// consecutive particles are compact (about 1.4 x 1.3 x 1.3 spacings on the
// lattice instead of 3.3 x 1.6 x 0.2): more of a group's evaluated pairs lie
// inside the support.  Steps between refreshes sort on the cell key alone
// (stable, so the cells keep the order of the last full sort).  Boundary
// particles take zeros there: a refresh never reorders them within a cell,
// so a fixed wall's particles keep their sorted positions through refreshes
// too (their groups only compute continuity, where compactness matters little).
constexpr int kSubBits = 2;
__host__ __device__ __forceinline__ uint32_t key_cell(uint32_t key) { return key >> kSubBits; }

// Cell coordinate along one axis and its half (see kSubBits).
__device__ __forceinline__ int axis_cell(double v, double o, double cs, int n, uint32_t &upper) {
    // floor((v - o) / cs) with an IEEE division, clamped to [0, n - 1]
    // (NaN -> 0).  Clamping is monotone, so pairs closer than cs still land
    // in adjacent cells.  upper: the position lies in the cell's upper half
    // (ordering only; 0 where clamped).
    const double t = (v - o) / cs;
    const double f = floor(t);
    upper = 0u;
    if (!(f >= 0.0)) return 0;
    if (f > (double)(n - 1)) return n - 1;
    upper = t - f >= 0.5 ? 1u : 0u;
    return (int)f;
}

// The sort key of a particle of instance ip at (x, y, z) (id: bit 31 =
// boundary).  Computed by the first sort pass from the positions, or by the
// update that produced them (the next step's keys).
__device__ __forceinline__ uint32_t sort_key(const Inst &ip, double x, double y, double z,
                                             uint32_t id) {
    uint32_t ux, uy, uz;
    const int cx = axis_cell(x, ip.ox, ip.cs, ip.nx, ux);
    const int cy = axis_cell(y, ip.oy, ip.cs, ip.ny, uy);
    const int cz = axis_cell(z, ip.oz, ip.cs, ip.nz, uz);
    const uint32_t lrow = (uint32_t)cz * (uint32_t)ip.ny + (uint32_t)cy;
    const uint32_t bnd = id >> 31;
    const uint32_t cell = half_row_key(ip, lrow, bnd) + (uint32_t)cx;
    return (cell << kSubBits) | (bnd ? 0u : (uy << 1) | ux);
}

// Device-side access to the instances: a table in the workspace (batches) or
// a single instance passed by value.
struct Insts {
    const Inst *tab;
    Inst one;
    int n;
    __device__ __forceinline__ Inst get(int k) const { return tab ? tab[k] : one; }
    // instance of an original particle id / global cell id
    __device__ __forceinline__ int of_id(uint32_t id) const {
        if (n == 1) return 0;
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tab[mid].pstart <= id) lo = mid; else hi = mid - 1;
        }
        return lo;
    }
    __device__ __forceinline__ int of_cell(uint32_t cell) const {
        if (n == 1) return 0;
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tab[mid].cell_base <= cell) lo = mid; else hi = mid - 1;
        }
        return lo;
    }
};

// Fixed walls in place.  While no boundary particle moves, the boundary
// particles of an instance keep their sorted positions from step to step
// (they follow all of the instance's fluid particles in key order, and their
// keys do not change), so the sort gives them the identity permutation and a
// step's gather may leave them where they are: it copies only what the
// update changed (the densities) and rewrites the density-dependent part of
// their view.
struct WallsInPlace {
    const unsigned int *walls;  // DevScalars::walls_move
    int allow;                  // the host allows it for this step
    // (the flag only changes inside an update, so every kernel of a step
    // gets the same answer)
    __device__ __forceinline__ bool on() const { return allow != 0 && *walls == 0u; }
};


// A problem: one or more instances sharing precision and particle arrays.
struct Problem {
    int precision = SPH_MIXED;
    int scheme = SPH_SCHEME_VERLET;  // sph_scheme, the same for every instance
    int64_t n = 0;          // particles in total
    int64_t ncells = 0;     // cells in total
    int64_t nrows = 0;      // rows in total
    std::vector<Inst> host; // host copy of the instance constants
    bool batch = false;     // table in the workspace (else single, by value)
};

// Byte offsets of the workspace regions (all 256-byte aligned).
struct WsLayout {
    int64_t n = 0;
    int64_t ncells = 0;
    int64_t nrows = 0;
    int64_t ntiles = 0;
    int64_t max_chunks = 0;
    int32_t ninst = 0;
    int32_t key_bits = 0;
    int32_t precision = 0;
    size_t keys = 0, keys_alt = 0, vals = 0, vals_alt = 0;
    size_t keys_next = 0;    // the next sort's input keys (written by the update)
    size_t sorted_keys = 0;  // where the sort leaves the keys (keys)
    size_t hist = 0;         // (digit, tile) counts of a sort pass
    size_t hist_off = 0;     // per digit, exclusive scan of its counts over the tiles
    size_t hist_tot = 0;     // per digit, its count over all tiles
    size_t scan_tot = 0;     // span totals of the chunks-per-half-row scan
    size_t row_cnt = 0;      // chunks per row
    size_t row_first = 0;    // first chunk of each row
    size_t cell_start = 0;
    size_t chunks = 0;
    size_t chunk_out = 0;    // ChunkOut per chunk
    size_t view0 = 0, view1 = 0, view2 = 0;
    size_t rates = 0;        // ax, ay, az, drho, mumax (each n values)
    size_t scalars = 0;
    size_t inst_tab = 0;     // Inst[ninst]
    size_t inst_state = 0;   // InstState[ninst]
    size_t diag_part = 0;
    size_t loads = 0;        // boundary-force partial sums: 4 doubles per cell row
    size_t impulse = 0;      // ImpulseState, then 2 x kMaxProbes doubles
    size_t total = 0;
    size_t view_elem = 0;    // bytes of one view record in the first array
    size_t rate_elem = 0;    // bytes of one rate value
};

WsLayout make_layout(const Problem &P);

// Typed views into a workspace.
struct Ws {
    WsLayout L;
    char *base = nullptr;
    template <class T>
    T *at(size_t off) const { return reinterpret_cast<T *>(base + off); }
    uint32_t *keys() const { return at<uint32_t>(L.keys); }
    uint32_t *keys_alt() const { return at<uint32_t>(L.keys_alt); }
    uint32_t *keys_next() const { return at<uint32_t>(L.keys_next); }
    uint32_t *vals() const { return at<uint32_t>(L.vals); }
    uint32_t *vals_alt() const { return at<uint32_t>(L.vals_alt); }
    uint32_t *hist() const { return at<uint32_t>(L.hist); }
    uint32_t *scan_tot() const { return at<uint32_t>(L.scan_tot); }
    uint32_t *row_first() const { return at<uint32_t>(L.row_first); }
    uint32_t *row_cnt() const { return at<uint32_t>(L.row_cnt); }
    uint32_t *hist_off() const { return at<uint32_t>(L.hist_off); }
    uint32_t *hist_tot() const { return at<uint32_t>(L.hist_tot); }
    uint32_t *cell_start() const { return at<uint32_t>(L.cell_start); }
    int4 *chunks() const { return at<int4>(L.chunks); }
    ChunkOut *chunk_out() const { return at<ChunkOut>(L.chunk_out); }
    DevScalars *scalars() const { return at<DevScalars>(L.scalars); }
    Inst *inst_tab() const { return at<Inst>(L.inst_tab); }
    InstState *inst_state() const { return at<InstState>(L.inst_state); }
    double *diag_part() const { return at<double>(L.diag_part); }
    double *loads() const { return at<double>(L.loads); }
    ImpulseState *impulse() const { return at<ImpulseState>(L.impulse); }
    double *impulse_sum() const { return at<double>(L.impulse + 256); }
    double *impulse_prev() const { return at<double>(L.impulse + 256) + kMaxProbes; }
};

// Accessor for the kernels of one call.
Insts insts_of(const Problem &P, const Ws &w);

// Thread-local error reporting.
int fail(int code, const std::string &msg);
int hip_check(hipError_t e, const char *what);
int launch_check(const char *what);

// Launchers implemented in the kernel translation units.
// What the previous step of a run leaves for the next sort: nothing, the keys
// of the current positions (a fused interaction that writes them), or the
// keys and their first-pass digit counts (the update kernel).
enum KeysLeft { kNoKeys = 0, kKeysOnly = 1, kKeysCounted = 2 };
int launch_sort(const Problem &P, const sph_state &s, const Ws &w, hipStream_t st, bool full,
                int keys, uint32_t **sorted_keys, uint32_t **perm);
// the fused interaction launched for P also writes the next sort's keys
bool fused_writes_keys(const Problem &P);
// exclusive scan of m values from `in` (left intact) to `out`; tot:
// ceil(m / kScanSpan) values of scratch
int launch_scan(const uint32_t *in, uint32_t *out, int64_t m, uint32_t *tot, hipStream_t st);
// walls_in_place: the two steps before gathered every particle, so this
// gather may leave fixed walls in place (WallsInPlace; the kernel decides
// from the device flag)
int launch_reorder(const Problem &P, sph_state &s, const Ws &w, const uint32_t *keys,
                   const uint32_t *perm, bool walls_in_place, hipStream_t st);
// steps of P may leave fixed walls in place (scheme and tuning)
bool walls_in_place_enabled(const Problem &P);
// lagged: also fix this step's dt from the previous interaction's bound (or dt > 0);
// zero_hist: also clear the sort's digit counts (w.hist())
int launch_chunks(const Problem &P, const Ws &w, bool lagged, double dt, hipStream_t st,
                  bool zero_hist = false);
// fuse: the interaction also advances every target (time update of step
// `step`) with the dt already stored per instance, instead of storing rates.
// after_kernel (optional): recorded between the interaction kernel and the
// per-instance reduction of its chunk records.
// count_shift >= 0 (fused, where fused_counts_digits): the update also adds
// the next sort's first-pass digit counts (from that bit) to w.hist(), which
// launch_chunks(zero_hist) cleared.
int launch_interact(const Problem &P, const sph_state &s, const Ws &w, hipStream_t st,
                    int32_t *st_nf = nullptr, int32_t *st_nb = nullptr,
                    uint32_t *st_hash = nullptr, bool fuse = false, int64_t step = 0,
                    hipEvent_t after_kernel = nullptr, int count_shift = -1);
// the fused interaction launched for P can also count the next sort's digits
bool fused_counts_digits(const Problem &P);
int launch_export_rates(const Problem &P, const Ws &w, double *ax, double *ay, double *az,
                        double *drho, double *mumax, hipStream_t st);
// hist_shift >= 0: the update also counts the digits (from that bit) of the
// keys it writes, per sort tile, for the first pass of the next step's sort.
int launch_integrate(const Problem &P, sph_state &s, const Ws &w, double dt, int64_t step,
                     hipStream_t st, int hist_shift = -1);
int launch_diag(const Problem &P, const sph_state &s, const Ws &w, const double *probes,
                int32_t np, sph_diag *out, double *probe_p, hipStream_t st);
// explicit MPS operators of instance 0 (outputs may be null)
int launch_mps(const Problem &P, const sph_state &s, const Ws &w, const sph_mps *m,
               const double *phi, double *pnd, double *lap, double *grad, double *sigma,
               int32_t *surface, hipStream_t st);
void mps_lattice_constants(double l0, double re, double *n0, double *lambda0);
// two-stage symplectic step: the predictor (rates at t in the workspace; fixes
// dt) or the corrector (rates at the predicted state)
int launch_symplectic(const Problem &P, sph_state &s, const Ws &w, double dt, bool corrector,
                      hipStream_t st);
// probe pressures (eq. sphpa) of instance 0 at np host points into the
// device array pout (np values); the points are staged in the workspace
int launch_probes(const Problem &P, const sph_state &s, const Ws &w, const double *probes,
                  int32_t np, double *pout, hipStream_t st);
// force on the boundary particles inside a box (instance 0), to the host
int launch_boundary_force(const Problem &P, const sph_state &s, const Ws &w, const double *box,
                          double *force, int64_t *count, hipStream_t st);
// probe pressures and their running impulse, to the host
int launch_probe_impulse(const Problem &P, const sph_state &s, const Ws &w, const double *probes,
                         int32_t np, int32_t reset, double *probe_p, double *impulse,
                         hipStream_t st);
int launch_set_density(const Problem &P, sph_state &s, const Ws &w, const double *rho,
                       int which, hipStream_t st);
int launch_get_density(const Problem &P, const sph_state &s, const Ws &w, double *rho,
                       int which, hipStream_t st);
int launch_ws_init(const Problem &P, const Ws &w, hipStream_t st);
void after_fused_step(sph_state &s);
int diag_blocks(int ninst);
int set_split(int precision, int split);
int set_group(int precision, int group);
int set_kernel(int precision, int kernel);
int set_xcd_run(int precision, int run);
void set_full_gather(int on);
int full_gather();
int split_for(const Problem &P);
int group_for(const Problem &P);
int kernel_for(const Problem &P);
int xcd_run_for(const Problem &P);
int chunk_for(const Problem &P);  // targets per chunk of the interaction launched for P

// Cell id layout inside an instance: local = cx + nx * (cy + ny * cz).
__host__ __device__ inline int64_t lin_cell(int cx, int cy, int cz, int nx, int ny) {
    return cx + (int64_t)nx * (cy + (int64_t)ny * cz);
}

}  // namespace wcsph
