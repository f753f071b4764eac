// extern "C" entry points of libwcsph: argument validation, workspace layout
// and the order of launches for each call.  Every argument is checked before
// anything is launched.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <algorithm>
#include <mutex>

#include "common.h"

namespace wcsph {

static thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return SPH_OK;
    return fail(SPH_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int launch_check(const char *what) { return hip_check(hipGetLastError(), what); }

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

WsLayout make_layout(const Problem &P) {
    WsLayout L;
    const int64_t n = P.n;
    L.n = n;
    L.precision = P.precision;
    L.ninst = (int32_t)P.host.size();
    L.ncells = P.ncells;
    L.nrows = P.nrows;
    L.ntiles = (n + sort_tile(n) - 1) / sort_tile(n);
    // at most ceil(particles / csz) + 1 chunks per half-row, csz >= kMinChunk
    L.max_chunks = (n + kMinChunk - 1) / kMinChunk + 4 * L.nrows;
    int bits = 0;
    while (bits < 32 && ((int64_t)1 << bits) < 2 * L.ncells) ++bits;
    L.key_bits = bits + kSubBits;
    const bool mixed = P.precision == SPH_MIXED;
    L.view_elem = mixed ? 16 : 32;
    L.rate_elem = mixed ? 4 : 8;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    L.keys = take(4 * (size_t)n);
    L.keys_alt = take(4 * (size_t)n);
    L.keys_next = take(4 * (size_t)n);
    L.vals = take(4 * (size_t)n);
    L.vals_alt = take(4 * (size_t)n);
    L.sorted_keys = L.keys;
    L.hist = take(4 * (size_t)kRadix * (size_t)L.ntiles);
    L.hist_off = take(4 * (size_t)kRadix * (size_t)L.ntiles);
    L.hist_tot = take(4 * (size_t)kRadix);
    L.scan_tot = take(4 * (((size_t)(2 * L.nrows) + kScanSpan - 1) / kScanSpan));
    L.row_cnt = take(4 * (size_t)(2 * L.nrows));  // per half-row
    L.row_first = take(4 * (size_t)(2 * L.nrows));
    L.cell_start = take(4 * (size_t)(2 * L.ncells + 1));
    L.chunks = take(sizeof(int4) * (size_t)L.max_chunks);
    L.chunk_out = take(sizeof(ChunkOut) * (size_t)L.max_chunks);
    L.view0 = take(L.view_elem * (size_t)n);
    L.view1 = take((mixed ? 8 : 32) * (size_t)n);
    L.view2 = take(16 * (size_t)n);
    L.rates = take(5 * L.rate_elem * (size_t)n);
    L.scalars = take(sizeof(DevScalars));
    L.inst_tab = take(sizeof(Inst) * (size_t)L.ninst);
    L.inst_state = take(sizeof(InstState) * (size_t)L.ninst);
    L.diag_part = take(sizeof(double) * ((size_t)L.ninst * diag_blocks(L.ninst) * kDiagFields +
                                         (size_t)L.ninst * kDiagFields + 4 * (size_t)kMaxProbes));
    L.loads = take(sizeof(double) * (4 * (size_t)L.nrows + 4));
    L.impulse = take(256 + sizeof(double) * 2 * (size_t)kMaxProbes);
    L.total = off;
    return L;
}

Insts insts_of(const Problem &P, const Ws &w) {
    Insts I;
    I.n = (int)P.host.size();
    I.one = P.host[0];
    I.tab = P.batch ? w.inst_tab() : nullptr;
    return I;
}

// Constants of one system occupying global cells from cell_base, rows from
// row_base and original ids [pstart, pend).
static Inst inst_from(const sph_params &p, uint32_t cell_base, uint32_t row_base,
                      uint32_t pstart, uint32_t pend) {
    Inst I{};
    I.ox = p.origin[0];
    I.oy = p.origin[1];
    I.oz = p.origin[2];
    I.cs = p.cell_size;
    I.h = p.h;
    I.invh = 1.0 / p.h;
    I.r2max = 4.0 * p.h * p.h;
    I.eta2 = p.eta2_coef * p.h * p.h;
    I.wd = 21.0 / (16.0 * M_PI * p.h * p.h * p.h);
    I.Fm = p.mass * 5.0 * I.wd / (p.h * p.h);
    I.alpha = p.alpha;
    I.kdelta = 2.0 * p.delta * p.h * p.c0;
    I.rho0 = p.rho0;
    I.c0 = p.c0;
    I.B = p.rho0 * p.c0 * p.c0 / p.gamma;
    I.gamma = p.gamma;
    I.gx = p.g[0];
    I.gy = p.g[1];
    I.gz = p.g[2];
    I.cfl = p.cfl;
    I.mass = p.mass;
    I.nx = p.dims[0];
    I.ny = p.dims[1];
    I.nz = p.dims[2];
    I.c_const = p.c_mode == SPH_C_CONST;
    I.delta_all = p.delta_pairs == SPH_DELTA_ALL;
    I.verlet_ns = p.verlet_ns;
    I.cell_base = cell_base;
    I.row_base = row_base;
    I.pstart = pstart;
    I.pend = pend;
    return I;
}

static Problem single_problem(const sph_params &p, int64_t n) {
    Problem P;
    P.precision = p.precision;
    P.scheme = p.scheme;
    P.n = n;
    P.ncells = (int64_t)p.dims[0] * p.dims[1] * p.dims[2];
    P.nrows = (int64_t)p.dims[1] * p.dims[2];
    P.host.push_back(inst_from(p, 0, 0, 0, (uint32_t)n));
    P.batch = false;
    return P;
}

static bool finite_all(std::initializer_list<double> v) {
    for (double d : v)
        if (!std::isfinite(d)) return false;
    return true;
}

static int check_params(const sph_params *p) {
    if (!p) return fail(SPH_E_INVAL, "params is NULL");
    if (!finite_all({p->dp, p->h, p->rho0, p->c0, p->gamma, p->alpha, p->delta, p->g[0], p->g[1],
                     p->g[2], p->eta2_coef, p->cfl, p->mass, p->origin[0], p->origin[1],
                     p->origin[2], p->cell_size}))
        return fail(SPH_E_INVAL, "non-finite parameter");
    if (!(p->dp > 0)) return fail(SPH_E_INVAL, "dp must be > 0");
    if (!(p->h > 0)) return fail(SPH_E_INVAL, "h must be > 0");
    if (!(p->rho0 > 0)) return fail(SPH_E_INVAL, "rho0 must be > 0");
    if (!(p->c0 > 0)) return fail(SPH_E_INVAL, "c0 must be > 0");
    if (!(p->gamma >= 1)) return fail(SPH_E_INVAL, "gamma must be >= 1");
    if (!(p->alpha >= 0)) return fail(SPH_E_INVAL, "alpha must be >= 0");
    if (!(p->delta >= 0 && p->delta <= 1)) return fail(SPH_E_INVAL, "delta must be in [0, 1]");
    if (!(p->eta2_coef >= 0)) return fail(SPH_E_INVAL, "eta2_coef must be >= 0");
    if (!(p->cfl > 0 && p->cfl <= 1)) return fail(SPH_E_INVAL, "cfl must be in (0, 1]");
    if (!(p->mass > 0)) return fail(SPH_E_INVAL, "mass must be > 0");
    if (!(p->cell_size >= 2.0 * p->h)) return fail(SPH_E_INVAL, "cell_size must be >= 2h");
    for (int k = 0; k < 3; ++k)
        if (p->dims[k] < 1) return fail(SPH_E_INVAL, "dims must be >= 1");
    const int64_t nc = (int64_t)p->dims[0] * p->dims[1] * p->dims[2];
    if (nc >= ((int64_t)1 << 29)) return fail(SPH_E_RANGE, "too many cells (>= 2^29)");
    if (p->precision != SPH_FP64 && p->precision != SPH_MIXED)
        return fail(SPH_E_INVAL, "unknown precision");
    if (p->c_mode != SPH_C_TAIT && p->c_mode != SPH_C_CONST)
        return fail(SPH_E_INVAL, "unknown c_mode");
    if (p->delta_pairs != SPH_DELTA_FLUID && p->delta_pairs != SPH_DELTA_ALL)
        return fail(SPH_E_INVAL, "unknown delta_pairs");
    if (p->scheme != SPH_SCHEME_VERLET && p->scheme != SPH_SCHEME_SYMPLECTIC)
        return fail(SPH_E_INVAL, "unknown scheme");
    return SPH_OK;
}

static int check_n(int64_t n) {
    if (n < 1) return fail(SPH_E_INVAL, "n must be >= 1");
    if (n >= ((int64_t)1 << 31)) return fail(SPH_E_RANGE, "n must be < 2^31");
    return SPH_OK;
}

static bool aligned(const void *ptr, size_t a) { return ((uintptr_t)ptr % a) == 0; }

static int check_state(int precision, const sph_state *s) {
    if (!s) return fail(SPH_E_INVAL, "state is NULL");
    if (int rc = check_n(s->n)) return rc;
    const void *ptrs[] = {s->x,      s->y,      s->z,      s->ux,      s->uy,      s->uz,
                          s->uxm,    s->uym,    s->uzm,    s->rho,     s->rhom,    s->id,
                          s->x_alt,  s->y_alt,  s->z_alt,  s->ux_alt,  s->uy_alt,  s->uz_alt,
                          s->uxm_alt, s->uym_alt, s->uzm_alt, s->rho_alt, s->rhom_alt, s->id_alt};
    for (const void *q : ptrs) {
        if (!q) return fail(SPH_E_INVAL, "state array pointer is NULL");
        if (!aligned(q, 4)) return fail(SPH_E_INVAL, "state array pointer is misaligned");
    }
    const double *d8[] = {s->x, s->y, s->z, s->ux, s->uy, s->uz, s->uxm, s->uym, s->uzm,
                          s->x_alt, s->y_alt, s->z_alt, s->ux_alt, s->uy_alt, s->uz_alt,
                          s->uxm_alt, s->uym_alt, s->uzm_alt};
    for (const double *q : d8)
        if (!aligned(q, 8)) return fail(SPH_E_INVAL, "double array pointer is misaligned");
    if (precision == SPH_FP64) {
        const void *r8[] = {s->rho, s->rhom, s->rho_alt, s->rhom_alt};
        for (const void *q : r8)
            if (!aligned(q, 8)) return fail(SPH_E_INVAL, "density pointer is misaligned");
    }
    if (s->reserved != 0) return fail(SPH_E_INVAL, "state reserved must be 0");
    return SPH_OK;
}

static int check_ws_ptr(const void *ws) {
    if (!ws) return fail(SPH_E_INVAL, "workspace is NULL");
    if (!aligned(ws, 256)) return fail(SPH_E_INVAL, "workspace must be 256-byte aligned");
    return SPH_OK;
}

// Single system: params + state + workspace -> problem and workspace view.
static int validate(const sph_params *p, const sph_state *s, void *ws, Problem *P, Ws *w) {
    if (int rc = check_params(p)) return rc;
    if (int rc = check_state(p->precision, s)) return rc;
    if (int rc = check_ws_ptr(ws)) return rc;
    *P = single_problem(*p, s->n);
    w->L = make_layout(*P);
    w->base = static_cast<char *>(ws);
    return SPH_OK;
}

// Batch description -> problem (host table of instances).
static int batch_problem(const sph_batch *b, Problem *P) {
    if (!b) return fail(SPH_E_INVAL, "batch is NULL");
    if (b->ninst < 1 || b->ninst > SPH_MAX_INSTANCES)
        return fail(SPH_E_INVAL, "ninst must be in [1, SPH_MAX_INSTANCES]");
    if (b->reserved != 0) return fail(SPH_E_INVAL, "batch reserved must be 0");
    if (!b->params || !b->counts) return fail(SPH_E_INVAL, "batch arrays are NULL");
    P->host.clear();
    P->batch = true;
    P->precision = b->params[0].precision;
    P->scheme = b->params[0].scheme;
    int64_t n = 0, cells = 0, rows = 0;
    for (int k = 0; k < b->ninst; ++k) {
        const sph_params &p = b->params[k];
        if (int rc = check_params(&p))
            return fail(rc, "instance " + std::to_string(k) + ": " + g_err);
        if (p.precision != P->precision)
            return fail(SPH_E_INVAL, "all instances must have the same precision");
        if (p.scheme != P->scheme)
            return fail(SPH_E_INVAL, "all instances must have the same scheme");
        const int64_t c = b->counts[k];
        if (c < 1) return fail(SPH_E_INVAL, "every instance needs >= 1 particle");
        const int64_t nc = (int64_t)p.dims[0] * p.dims[1] * p.dims[2];
        const int64_t nr = (int64_t)p.dims[1] * p.dims[2];
        if (n + c >= ((int64_t)1 << 31)) return fail(SPH_E_RANGE, "total particles must be < 2^31");
        if (cells + nc >= ((int64_t)1 << 29))
            return fail(SPH_E_RANGE, "total cells must be < 2^29");
        P->host.push_back(inst_from(p, (uint32_t)cells, (uint32_t)rows, (uint32_t)n,
                                    (uint32_t)(n + c)));
        n += c;
        cells += nc;
        rows += nr;
    }
    P->n = n;
    P->ncells = cells;
    P->nrows = rows;
    return SPH_OK;
}

static int validate_batch(const sph_batch *b, const sph_state *s, void *ws, Problem *P, Ws *w) {
    if (int rc = batch_problem(b, P)) return rc;
    if (int rc = check_state(P->precision, s)) return rc;
    if (s->n != P->n) return fail(SPH_E_INVAL, "state n must equal the sum of the counts");
    if (int rc = check_ws_ptr(ws)) return rc;
    w->L = make_layout(*P);
    w->base = static_cast<char *>(ws);
    return SPH_OK;
}

// Timing marks: events recorded around one region of a step.
struct Marks {
    int region = SPH_REGION_INTERACT;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int at(int r, bool begin, hipStream_t st) const {
        if (!e0 || r != region) return SPH_OK;
        return hip_check(hipEventRecord(begin ? e0 : e1, st), "event record");
    }
};

// full: sort on the sub-cell bits too (see kSubBits); the steps between
// refreshes sort on the cell key alone.  keys (KeysLeft): what the previous
// step of this same run left (else the keys and counts are computed from the
// positions here).
// walls_in_place: the previous two steps of this call gathered every
// particle, so this gather may leave fixed walls in place (WallsInPlace).
// zero_hist: the step's fused interaction counts the next sort's digits.
static int build_cells(const Problem &P, sph_state &s, const Ws &w, hipStream_t st,
                       bool lagged = false, double dt = 0.0, const Marks &m = Marks(),
                       bool full = true, int keys = kNoKeys, bool walls_in_place = false,
                       bool zero_hist = false) {
    if (int rc = m.at(SPH_REGION_STEP, true, st)) return rc;
    uint32_t *sorted = nullptr, *perm = nullptr;
    if (int rc = m.at(SPH_REGION_SORT, true, st)) return rc;
    if (int rc = launch_sort(P, s, w, st, full, keys, &sorted, &perm)) return rc;
    if (int rc = m.at(SPH_REGION_SORT, false, st)) return rc;
    if (int rc = m.at(SPH_REGION_REORDER, true, st)) return rc;
    if (int rc = launch_reorder(P, s, w, sorted, perm, walls_in_place, st)) return rc;
    if (int rc = m.at(SPH_REGION_REORDER, false, st)) return rc;
    if (int rc = launch_chunks(P, w, lagged, dt, st, zero_hist)) return rc;
    s.cells_valid = 1;
    return SPH_OK;
}

static int64_t graph_period(const Problem &P);

// Steps whose cell list sorts on every key bit: multiples of this period (the
// graph period when there is one, so that a replayed graph refreshes at the
// same steps as eager launches would).
static int64_t refresh_period(const Problem &P) {
    const int64_t L = graph_period(P);
    return L > 0 ? L : 40;
}

// One step of the two-stage symplectic scheme: cells and rates at t, the
// predictor (which fixes dt), cells and rates at the predicted state, the
// corrector.  The cell lists compute their keys from the positions.
static int symplectic_step(const Problem &P, sph_state &s, const Ws &w, double dt, int64_t step,
                           hipStream_t st, const Marks &m) {
    if (!s.cells_valid) {
        const bool full = step % refresh_period(P) == 0;
        if (int rc = build_cells(P, s, w, st, false, dt, m, full, kNoKeys)) return rc;
    } else {
        if (int rc = m.at(SPH_REGION_STEP, true, st)) return rc;
        if (int rc = launch_chunks(P, w, false, dt, st)) return rc;
    }
    if (int rc = m.at(SPH_REGION_INTERACT, true, st)) return rc;
    hipEvent_t after = (m.region == SPH_REGION_INTERACT && m.e0) ? m.e1 : nullptr;
    if (int rc = launch_interact(P, s, w, st, nullptr, nullptr, nullptr, false, step, after))
        return rc;
    if (int rc = launch_symplectic(P, s, w, dt, false, st)) return rc;
    s.cells_valid = 0;
    if (int rc = build_cells(P, s, w, st, false, dt, Marks(), false, kNoKeys)) return rc;
    if (int rc = launch_interact(P, s, w, st)) return rc;
    if (int rc = launch_symplectic(P, s, w, dt, true, st)) return rc;
    if (int rc = m.at(SPH_REGION_STEP, false, st)) return rc;
    s.cells_valid = 0;
    return SPH_OK;
}

// Whether step k of this call may leave fixed walls in place.  The boundary
// particles must already sit, in both buffers of the state, at the positions
// this step's sort gives them (refreshes included: boundary keys carry no
// sub-cell bits), so the call's first two steps gather every particle.
static bool walls_in_place_at(const Problem &P, int64_t k) {
    return k >= 2 && walls_in_place_enabled(P);
}

// One step.  fused: the lagged-dt form, where the interaction also advances
// the state (one kernel instead of interaction + update).  k: the step's
// index within this call.
static int one_step(const Problem &P, sph_state &s, const Ws &w, double dt, int64_t step,
                    bool fused, hipStream_t st, const Marks &m = Marks(), int keys = kNoKeys,
                    int64_t k = 0) {
    if (P.scheme == SPH_SCHEME_SYMPLECTIC) return symplectic_step(P, s, w, dt, step, st, m);
    // the next step's sort: on every key bit at a refresh, else from kSubBits;
    // a fused interaction that writes its keys may also count its first digits
    const int next_low = (step + 1) % refresh_period(P) == 0 ? 0 : kSubBits;
    const bool count = fused && fused_counts_digits(P);
    if (!s.cells_valid) {
        const bool full = step % refresh_period(P) == 0;
        if (int rc = build_cells(P, s, w, st, fused, dt, m, full, keys, walls_in_place_at(P, k),
                                 count))
            return rc;
    } else {
        if (int rc = m.at(SPH_REGION_STEP, true, st)) return rc;
        if (int rc = launch_chunks(P, w, fused, dt, st, count)) return rc;  // fresh dt bound
    }
    // the interaction region ends with the kernel (before the reduction of
    // its chunk records)
    if (int rc = m.at(SPH_REGION_INTERACT, true, st)) return rc;
    hipEvent_t after = m.region == SPH_REGION_INTERACT ? m.e1 : nullptr;
    if (!m.e0) after = nullptr;
    if (int rc = launch_interact(P, s, w, st, nullptr, nullptr, nullptr, fused, step, after,
                                 count ? next_low : -1))
        return rc;
    if (fused) {
        after_fused_step(s);
    } else {
        // the update also counts the first digits of the next step's sort
        if (int rc = launch_integrate(P, s, w, dt, step, st, next_low)) return rc;
    }
    if (int rc = m.at(SPH_REGION_STEP, false, st)) return rc;
    s.cells_valid = 0;
    return SPH_OK;
}

// What a step leaves for the next sort (KeysLeft): the update kernel writes
// the keys and counts their first digits; a fused interaction may write the
// keys, and the row-split one with them count their first digits too.
static int keys_after(const Problem &P, bool fused) {
    if (P.scheme == SPH_SCHEME_SYMPLECTIC) return kNoKeys;
    if (!fused || fused_counts_digits(P)) return kKeysCounted;
    return fused_writes_keys(P) ? kKeysOnly : kNoKeys;
}

static int64_t gcd64(int64_t a, int64_t b) {
    while (b) {
        const int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// Steps after which a captured sequence repeats itself: the state pointers
// cycle with period 4 (the cell-order gather and the level rotation each
// swap pairs of buffers), and each instance's Euler reset with its N_s.
static int64_t graph_period(const Problem &P) {
    int64_t L = 4;
    for (const Inst &ip : P.host) {
        if (ip.verlet_ns > 0) L = L / gcd64(L, ip.verlet_ns) * ip.verlet_ns;
        if (L > kMaxGraphSteps) return 0;
    }
    return L;
}

static bool same_pointers(const sph_state &a, const sph_state &b) {
    return a.x == b.x && a.y == b.y && a.z == b.z && a.ux == b.ux && a.uy == b.uy &&
           a.uz == b.uz && a.uxm == b.uxm && a.uym == b.uym && a.uzm == b.uzm &&
           a.rho == b.rho && a.rhom == b.rhom && a.id == b.id && a.x_alt == b.x_alt &&
           a.y_alt == b.y_alt && a.z_alt == b.z_alt && a.ux_alt == b.ux_alt &&
           a.uy_alt == b.uy_alt && a.uz_alt == b.uz_alt && a.uxm_alt == b.uxm_alt &&
           a.uym_alt == b.uym_alt && a.uzm_alt == b.uzm_alt && a.rho_alt == b.rho_alt &&
           a.rhom_alt == b.rhom_alt && a.id_alt == b.id_alt;
}

// Capture `len` steps from index step into a graph (nothing runs), then
// replay it `reps` times.  The state pointers must come back to where they
// started, which the period guarantees.
static int graph_steps(const Problem &P, sph_state &s, const Ws &w, double dt, int64_t step,
                       int64_t len, int64_t reps, bool lagged, hipStream_t st, int64_t k0) {
    const sph_state s0 = s;
    if (int rc = hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed), "capture"))
        return rc;
    int rc = SPH_OK;
    // the first captured step computes its keys from the positions (a replay
    // may follow anything); the later ones take what the step before left.
    // k0: the index of the first captured step within the call.
    for (int64_t k = 0; k < len && rc == SPH_OK; ++k)
        rc = one_step(P, s, w, dt, step + k, lagged && step + k > 0, st, Marks(),
                      k > 0 ? keys_after(P, lagged && step + k - 1 > 0) : kNoKeys,
                      k0 + k);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(st, &g);
    if (rc == SPH_OK) rc = hip_check(ec, "end capture");
    if (rc == SPH_OK && !same_pointers(s, s0))
        rc = fail(SPH_E_STATE, "captured steps did not return the state to its buffers");
    hipGraphExec_t ex = nullptr;
    if (rc == SPH_OK)
        rc = hip_check(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0), "graph instantiate");
    for (int64_t r = 0; r < reps && rc == SPH_OK; ++r)
        rc = hip_check(hipGraphLaunch(ex, st), "graph launch");
    if (ex) {
        // the replays must finish before the executable graph goes away
        const int rs = hip_check(hipStreamSynchronize(st), "graph sync");
        if (rc == SPH_OK) rc = rs;
        (void)hipGraphExecDestroy(ex);
    }
    if (g) (void)hipGraphDestroy(g);
    s = s0;
    s.cells_valid = 0;
    return rc;
}

static int run_steps(const Problem &P, sph_state &s, const Ws &w, int64_t nsteps, double dt,
                     int64_t step0, int mode, hipStream_t st, int region = SPH_REGION_INTERACT,
                     void *const *ev_begin = nullptr, void *const *ev_end = nullptr) {
    const bool lagged = (mode & SPH_RUN_LAGGED) != 0;
    const int64_t L = (mode & SPH_RUN_GRAPH) ? graph_period(P) : 0;
    int64_t k = 0;
    // the first step of a call computes its keys from the positions (the
    // caller may have moved particles); later steps take what the previous
    // step left
    int keys = kNoKeys;
    while (k < nsteps) {
        const int64_t idx = step0 + k;
        // graphs of L steps from the call's third step on (after the two steps
        // that gather every particle): the step-dependent choices (Euler
        // reset, refresh) and the buffers repeat with period L from any step
        if (L > 0 && k >= 2 && nsteps - k >= L && !ev_begin) {
            const int64_t reps = (nsteps - k) / L;
            s.cells_valid = 0;  // every captured step rebuilds its cells
            if (int rc = graph_steps(P, s, w, dt, idx, L, reps, lagged, st, k)) return rc;
            k += reps * L;
            keys = keys_after(P, lagged);  // the graph's last step has index > 0
            continue;
        }
        Marks m;
        m.region = region;
        if (ev_begin) {
            m.e0 = static_cast<hipEvent_t>(ev_begin[k]);
            m.e1 = static_cast<hipEvent_t>(ev_end[k]);
        }
        if (int rc = one_step(P, s, w, dt, idx, lagged && idx > 0, st, m, keys, k)) return rc;
        keys = keys_after(P, lagged && idx > 0);
        ++k;
    }
    return SPH_OK;
}

static int check_run_args(double dt, int64_t nsteps, int64_t step0, int mode) {
    if (!std::isfinite(dt)) return fail(SPH_E_INVAL, "dt must be finite");
    if (nsteps < 0 || step0 < 0) return fail(SPH_E_INVAL, "nsteps and step0 must be >= 0");
    if (mode & ~(SPH_RUN_LAGGED | SPH_RUN_GRAPH)) return fail(SPH_E_INVAL, "unknown mode bits");
    return SPH_OK;
}

static int check_events(int64_t nsteps, int32_t region, void *const *ev_begin,
                        void *const *ev_end) {
    if (region < SPH_REGION_INTERACT || region > SPH_REGION_STEP)
        return fail(SPH_E_INVAL, "unknown region");
    if ((ev_begin == nullptr) != (ev_end == nullptr))
        return fail(SPH_E_INVAL, "ev_begin and ev_end must both be given or both be NULL");
    if (ev_begin)
        for (int64_t k = 0; k < nsteps; ++k)
            if ((ev_begin[k] == nullptr) != (ev_end[k] == nullptr))
                return fail(SPH_E_INVAL, "event handles of a step must both be set or both NULL");
    return SPH_OK;
}

static int check_rates_out(const double *ax, const double *ay, const double *az,
                           const double *drho, const double *mumax) {
    if (!ax || !ay || !az || !drho) return fail(SPH_E_INVAL, "output pointer is NULL");
    const double *outs[] = {ax, ay, az, drho};
    for (const double *q : outs)
        if (!aligned(q, 8)) return fail(SPH_E_INVAL, "output pointer is misaligned");
    if (mumax && !aligned(mumax, 8)) return fail(SPH_E_INVAL, "mumax is misaligned");
    return SPH_OK;
}

static int interact_rates(const Problem &P, const sph_state &s, const Ws &w, double *ax,
                          double *ay, double *az, double *drho, double *mumax, hipStream_t st) {
    if (!s.cells_valid) return fail(SPH_E_STATE, "rates need current cells (build_cells)");
    if (int rc = launch_chunks(P, w, false, 0.0, st)) return rc;  // resets the dt bound
    if (int rc = launch_interact(P, s, w, st)) return rc;
    return launch_export_rates(P, w, ax, ay, az, drho, mumax, st);
}

static int ws_init(const Problem &P, void *ws, size_t ws_bytes, hipStream_t st) {
    if (int rc = check_ws_ptr(ws)) return rc;
    Ws w;
    w.L = make_layout(P);
    w.base = static_cast<char *>(ws);
    if (ws_bytes < w.L.total) return fail(SPH_E_SIZE, "workspace too small");
    return launch_ws_init(P, w, st);
}

static int density_io(const Problem &P, sph_state *s, const Ws &w, double *rho, int32_t which,
                      bool set, hipStream_t st) {
    if (!rho || !aligned(rho, 8)) return fail(SPH_E_INVAL, "rho is NULL or misaligned");
    if (which != 0 && which != 1) return fail(SPH_E_INVAL, "which must be 0 or 1");
    return set ? launch_set_density(P, *s, w, rho, which, st)
               : launch_get_density(P, *s, w, rho, which, st);
}

// ------------------------------------------------------- no-alloc scratch
//
// sph_run_noalloc's workspace: a file-scope device array, of which every GPU
// the library runs on holds its own copy for the life of the process.  Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): scratch_base() asks the runtime for the array's
// device address once per device, with that device current, and every later
// use goes through that address.
static __device__ __align__(256) unsigned char scratch[SPH_NOALLOC_WS_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_addr[kMaxDevices] = {};

// Device of the stream (the current device for the null stream).
static int stream_device(hipStream_t st, int *dev) {
    if (st) return hip_check(hipStreamGetDevice(st, dev), "stream device");
    return hip_check(hipGetDevice(dev), "current device");
}

static int scratch_base(hipStream_t st, char **base) {
    int dev = 0;
    if (int rc = stream_device(st, &dev)) return rc;
    if (dev < 0 || dev >= kMaxDevices) return fail(SPH_E_HIP, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        int cur = 0;
        if (int rc = hip_check(hipGetDevice(&cur), "current device")) return rc;
        if (cur != dev)
            if (int rc = hip_check(hipSetDevice(dev), "select the stream's device")) return rc;
        void *addr = nullptr;
        const int rc = hip_check(hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch)),
                                 "scratch symbol address");
        if (cur != dev) (void)hipSetDevice(cur);
        if (rc) return rc;
        if (!addr) return fail(SPH_E_HIP, "scratch symbol address is NULL");
        g_scratch_addr[dev] = addr;
    }
    *base = static_cast<char *>(g_scratch_addr[dev]);
    return SPH_OK;
}

}  // namespace wcsph

using namespace wcsph;

extern "C" {

int sph_version(void) { return SPH_ABI_VERSION; }

const char *sph_last_error(void) { return g_err.c_str(); }

int sph_check_params(const sph_params *p) { return check_params(p); }

int sph_set_tuning(const sph_tuning *t) {
    if (!t) return fail(SPH_E_INVAL, "tuning is NULL");
    auto split_ok = [](int v) { return v == 0 || v == 1 || v == 3 || v == 9; };
    auto group_ok = [](int v) { return v == 0 || v == 8 || v == 16 || v == 64; };
    auto kernel_ok = [](int v) {
        return v == SPH_KERNEL_AUTO || v == SPH_KERNEL_ROWS || v == SPH_KERNEL_GROUPS ||
               v == SPH_KERNEL_COOP || v == SPH_KERNEL_COOP2;
    };
    if (!split_ok(t->split_fp64) || !split_ok(t->split_mixed))
        return fail(SPH_E_INVAL, "split must be 0, 1, 3 or 9");
    if (!group_ok(t->group_fp64) || !group_ok(t->group_mixed))
        return fail(SPH_E_INVAL, "group must be 0, 8, 16 or 64");
    if (!kernel_ok(t->kernel_fp64) || !kernel_ok(t->kernel_mixed))
        return fail(SPH_E_INVAL, "kernel must be an sph_kernel value");
    auto run_ok = [](int v) { return v == 0 || v == 1 || v == 8 || v == 32; };
    if (!run_ok(t->xcd_run_fp64) || !run_ok(t->xcd_run_mixed))
        return fail(SPH_E_INVAL, "xcd_run must be 0, 1, 8 or 32");
    if (t->full_gather != 0 && t->full_gather != 1)
        return fail(SPH_E_INVAL, "full_gather must be 0 or 1");
    set_split(SPH_FP64, t->split_fp64);
    set_split(SPH_MIXED, t->split_mixed);
    set_group(SPH_FP64, t->group_fp64);
    set_group(SPH_MIXED, t->group_mixed);
    set_kernel(SPH_FP64, t->kernel_fp64);
    set_kernel(SPH_MIXED, t->kernel_mixed);
    set_xcd_run(SPH_FP64, t->xcd_run_fp64);
    set_xcd_run(SPH_MIXED, t->xcd_run_mixed);
    set_full_gather(t->full_gather);
    return SPH_OK;
}

int sph_get_split(const sph_params *p, int64_t n, int32_t *split, int32_t *group,
                  int32_t *kernel) {
    if (int rc = check_params(p)) return rc;
    if (int rc = check_n(n)) return rc;
    if (!split || !group || !kernel) return fail(SPH_E_INVAL, "output is NULL");
    const Problem P = single_problem(*p, n);
    *split = split_for(P);
    *group = group_for(P);
    *kernel = kernel_for(P);
    return SPH_OK;
}

int sph_workspace_bytes(const sph_params *p, int64_t n, size_t *bytes) {
    if (int rc = check_params(p)) return rc;
    if (int rc = check_n(n)) return rc;
    if (!bytes) return fail(SPH_E_INVAL, "bytes is NULL");
    *bytes = make_layout(single_problem(*p, n)).total;
    return SPH_OK;
}

int sph_workspace_init(const sph_params *p, int64_t n, void *ws, size_t ws_bytes, void *stream) {
    if (int rc = check_params(p)) return rc;
    if (int rc = check_n(n)) return rc;
    return ws_init(single_problem(*p, n), ws, ws_bytes, static_cast<hipStream_t>(stream));
}

int sph_set_density(const sph_params *p, sph_state *s, const double *rho, int32_t which,
                    void *stream) {
    if (int rc = check_params(p)) return rc;
    if (int rc = check_state(p->precision, s)) return rc;
    const Problem P = single_problem(*p, s->n);
    Ws w;  // single systems need no workspace for the conversion
    return density_io(P, s, w, const_cast<double *>(rho), which, true,
                      static_cast<hipStream_t>(stream));
}

int sph_get_density(const sph_params *p, const sph_state *s, double *rho, int32_t which,
                    void *stream) {
    if (int rc = check_params(p)) return rc;
    if (int rc = check_state(p->precision, s)) return rc;
    const Problem P = single_problem(*p, s->n);
    Ws w;
    return density_io(P, const_cast<sph_state *>(s), w, rho, which, false,
                      static_cast<hipStream_t>(stream));
}

int sph_build_cells(const sph_params *p, sph_state *s, void *ws, void *stream) {
    Problem P;
    Ws w;
    if (int rc = validate(p, s, ws, &P, &w)) return rc;
    return build_cells(P, *s, w, static_cast<hipStream_t>(stream));
}

int sph_interact(const sph_params *p, const sph_state *s, void *ws, double *ax, double *ay,
                 double *az, double *drho, double *mumax, void *stream) {
    Problem P;
    Ws w;
    if (int rc = validate(p, s, ws, &P, &w)) return rc;
    if (int rc = check_rates_out(ax, ay, az, drho, mumax)) return rc;
    return interact_rates(P, *s, w, ax, ay, az, drho, mumax, static_cast<hipStream_t>(stream));
}

int sph_neighbour_stats(const sph_params *p, const sph_state *s, void *ws, int32_t *n_fluid_nbrs,
                        int32_t *n_boundary_nbrs, uint32_t *id_hash, void *stream) {
    Problem P;
    Ws w;
    if (int rc = validate(p, s, ws, &P, &w)) return rc;
    if (!n_fluid_nbrs || !n_boundary_nbrs || !id_hash)
        return fail(SPH_E_INVAL, "output pointer is NULL");
    if (!aligned(n_fluid_nbrs, 4) || !aligned(n_boundary_nbrs, 4) || !aligned(id_hash, 4))
        return fail(SPH_E_INVAL, "output pointer is misaligned");
    if (!s->cells_valid) return fail(SPH_E_STATE, "sph_neighbour_stats needs current cells");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (int rc = launch_chunks(P, w, false, 0.0, st)) return rc;
    return launch_interact(P, *s, w, st, n_fluid_nbrs, n_boundary_nbrs, id_hash);
}

int sph_step(const sph_params *p, sph_state *s, void *ws, double dt, int64_t step_index,
             void *stream) {
    Problem P;
    Ws w;
    if (int rc = validate(p, s, ws, &P, &w)) return rc;
    if (int rc = check_run_args(dt, 1, step_index, 0)) return rc;
    return one_step(P, *s, w, dt, step_index, false, static_cast<hipStream_t>(stream));
}

int sph_run(const sph_params *p, sph_state *s, void *ws, int64_t nsteps, double dt, int64_t step0,
            void *stream) {
    Problem P;
    Ws w;
    if (int rc = validate(p, s, ws, &P, &w)) return rc;
    if (int rc = check_run_args(dt, nsteps, step0, 0)) return rc;
    return run_steps(P, *s, w, nsteps, dt, step0, 0, static_cast<hipStream_t>(stream));
}

int sph_run_profiled(const sph_params *p, sph_state *s, void *ws, int64_t nsteps, double dt,
                     int64_t step0, int32_t region, void *const *ev_begin, void *const *ev_end,
                     void *stream) {
    Problem P;
    Ws w;
    if (int rc = validate(p, s, ws, &P, &w)) return rc;
    if (int rc = check_run_args(dt, nsteps, step0, 0)) return rc;
    if (int rc = check_events(nsteps, region, ev_begin, ev_end)) return rc;
    return run_steps(P, *s, w, nsteps, dt, step0, 0, static_cast<hipStream_t>(stream), region,
                     ev_begin, ev_end);
}

int sph_run_noalloc(const sph_params *p, sph_state *s, int64_t nsteps, double dt, int64_t step0,
                    void *stream) {
    if (int rc = check_params(p)) return rc;
    if (int rc = check_state(p->precision, s)) return rc;
    if (int rc = check_run_args(dt, nsteps, step0, 0)) return rc;
    const Problem P = single_problem(*p, s->n);
    Ws w;
    w.L = make_layout(P);
    if (w.L.total > (size_t)SPH_NOALLOC_WS_BYTES)
        return fail(SPH_E_SIZE, "sph_run_noalloc: the problem needs " + std::to_string(w.L.total) +
                                    " bytes of workspace, the static scratch holds " +
                                    std::to_string((size_t)SPH_NOALLOC_WS_BYTES));
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (int rc = scratch_base(st, &w.base)) return rc;
    // the scratch keeps whatever the last call left: restart the clock and
    // counters (a kernel, no memset), and rebuild the cell list from the
    // state's positions
    if (int rc = launch_ws_init(P, w, st)) return rc;
    s->cells_valid = 0;
    return run_steps(P, *s, w, nsteps, dt, step0, 0, st);
}

int sph_diagnostics(const sph_params *p, const sph_state *s, void *ws, const double *probes_xyz,
                    int32_t np, sph_diag *out, double *probe_p, void *stream) {
    Problem P;
    Ws w;
    if (int rc = validate(p, s, ws, &P, &w)) return rc;
    if (!out) return fail(SPH_E_INVAL, "out is NULL");
    if (np < 0 || np > kMaxProbes) return fail(SPH_E_INVAL, "np must be in [0, 1024]");
    if (np > 0 && (!probes_xyz || !probe_p)) return fail(SPH_E_INVAL, "probe arrays are NULL");
    if (!s->cells_valid) return fail(SPH_E_STATE, "sph_diagnostics needs current cells");
    return launch_diag(P, *s, w, probes_xyz, np, out, probe_p, static_cast<hipStream_t>(stream));
}

int sph_boundary_force(const sph_params *p, const sph_state *s, void *ws, const double *box,
                       double *force, int64_t *count, void *stream) {
    Problem P;
    Ws w;
    if (int rc = validate(p, s, ws, &P, &w)) return rc;
    if (!box || !force) return fail(SPH_E_INVAL, "box and force must not be NULL");
    for (int k = 0; k < 3; ++k) {
        if (!std::isfinite(box[2 * k]) || !std::isfinite(box[2 * k + 1]))
            return fail(SPH_E_INVAL, "box must be finite");
        if (!(box[2 * k] <= box[2 * k + 1])) return fail(SPH_E_INVAL, "box needs lo <= hi");
    }
    if (!s->cells_valid) return fail(SPH_E_STATE, "sph_boundary_force needs current cells");
    return launch_boundary_force(P, *s, w, box, force, count, static_cast<hipStream_t>(stream));
}

int sph_probe_impulse(const sph_params *p, const sph_state *s, void *ws, const double *probes_xyz,
                      int32_t np, int32_t reset, double *probe_p, double *impulse, void *stream) {
    Problem P;
    Ws w;
    if (int rc = validate(p, s, ws, &P, &w)) return rc;
    if (np < 1 || np > kMaxProbes) return fail(SPH_E_INVAL, "np must be in [1, 1024]");
    if (!probes_xyz || !probe_p || !impulse) return fail(SPH_E_INVAL, "probe arrays are NULL");
    if (reset != 0 && reset != 1) return fail(SPH_E_INVAL, "reset must be 0 or 1");
    for (int k = 0; k < 3 * np; ++k)
        if (!std::isfinite(probes_xyz[k])) return fail(SPH_E_INVAL, "probe points must be finite");
    if (!s->cells_valid) return fail(SPH_E_STATE, "sph_probe_impulse needs current cells");
    return launch_probe_impulse(P, *s, w, probes_xyz, np, reset, probe_p, impulse,
                                static_cast<hipStream_t>(stream));
}

int sph_mps_constants(double l0, double re, double *n0, double *lambda0) {
    if (!n0 || !lambda0) return fail(SPH_E_INVAL, "outputs must not be NULL");
    if (!(std::isfinite(l0) && l0 > 0.0)) return fail(SPH_E_INVAL, "l0 must be > 0");
    if (!(std::isfinite(re) && re > 0.0 && re <= 64.0 * l0))
        return fail(SPH_E_INVAL, "re must be in (0, 64 l0]");
    mps_lattice_constants(l0, re, n0, lambda0);
    if (!(*n0 > 0.0)) return fail(SPH_E_INVAL, "no lattice point within re");
    return SPH_OK;
}

int sph_mps_operators(const sph_params *p, const sph_state *s, void *ws, const sph_mps *m,
                      const double *phi, double *pnd, double *lap, double *grad, double *sigma,
                      int32_t *surface, void *stream) {
    Problem P;
    Ws w;
    if (int rc = validate(p, s, ws, &P, &w)) return rc;
    if (!m) return fail(SPH_E_INVAL, "mps parameters are NULL");
    if (!finite_all({m->re, m->n0, m->lambda0, m->beta1, m->rho1, m->l0}))
        return fail(SPH_E_INVAL, "non-finite mps parameter");
    if (!(m->re > 0.0)) return fail(SPH_E_INVAL, "re must be > 0");
    if (!(m->re <= p->cell_size)) return fail(SPH_E_INVAL, "re must not exceed the cell size");
    if (!(m->n0 > 0.0) || !(m->lambda0 > 0.0))
        return fail(SPH_E_INVAL, "n0 and lambda0 must be > 0");
    if (!(m->beta1 > 0.0 && m->beta1 <= 1.0)) return fail(SPH_E_INVAL, "beta1 must be in (0, 1]");
    if (!(m->rho1 >= 0.0) || !(m->l0 > 0.0))
        return fail(SPH_E_INVAL, "rho1 must be >= 0 and l0 > 0");
    if (!phi && (lap || grad)) return fail(SPH_E_INVAL, "lap and grad need phi");
    const void *ptrs[] = {phi, pnd, lap, grad, sigma};
    for (const void *q : ptrs)
        if (q && !aligned(q, 8)) return fail(SPH_E_INVAL, "mps array is misaligned");
    if (surface && !aligned(surface, 4)) return fail(SPH_E_INVAL, "surface is misaligned");
    if (!s->cells_valid) return fail(SPH_E_STATE, "sph_mps_operators needs current cells");
    return launch_mps(P, *s, w, m, phi, pnd, lap, grad, sigma, surface,
                      static_cast<hipStream_t>(stream));
}

// ------------------------------------------------------------------ batch

int sph_batch_workspace_bytes(const sph_batch *b, size_t *bytes) {
    Problem P;
    if (int rc = batch_problem(b, &P)) return rc;
    if (!bytes) return fail(SPH_E_INVAL, "bytes is NULL");
    *bytes = make_layout(P).total;
    return SPH_OK;
}

int sph_batch_workspace_init(const sph_batch *b, void *ws, size_t ws_bytes, void *stream) {
    Problem P;
    if (int rc = batch_problem(b, &P)) return rc;
    return ws_init(P, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

int sph_batch_set_density(const sph_batch *b, sph_state *s, void *ws, const double *rho,
                          int32_t which, void *stream) {
    Problem P;
    Ws w;
    if (int rc = validate_batch(b, s, ws, &P, &w)) return rc;
    return density_io(P, s, w, const_cast<double *>(rho), which, true,
                      static_cast<hipStream_t>(stream));
}

int sph_batch_get_density(const sph_batch *b, const sph_state *s, void *ws, double *rho,
                          int32_t which, void *stream) {
    Problem P;
    Ws w;
    if (int rc = validate_batch(b, s, ws, &P, &w)) return rc;
    return density_io(P, const_cast<sph_state *>(s), w, rho, which, false,
                      static_cast<hipStream_t>(stream));
}

int sph_batch_build_cells(const sph_batch *b, sph_state *s, void *ws, void *stream) {
    Problem P;
    Ws w;
    if (int rc = validate_batch(b, s, ws, &P, &w)) return rc;
    return build_cells(P, *s, w, static_cast<hipStream_t>(stream));
}

int sph_batch_interact(const sph_batch *b, const sph_state *s, void *ws, double *ax, double *ay,
                       double *az, double *drho, double *mumax, void *stream) {
    Problem P;
    Ws w;
    if (int rc = validate_batch(b, s, ws, &P, &w)) return rc;
    if (int rc = check_rates_out(ax, ay, az, drho, mumax)) return rc;
    return interact_rates(P, *s, w, ax, ay, az, drho, mumax, static_cast<hipStream_t>(stream));
}

int sph_batch_run(const sph_batch *b, sph_state *s, void *ws, int64_t nsteps, double dt,
                  int64_t step0, int32_t mode, void *stream) {
    Problem P;
    Ws w;
    if (int rc = validate_batch(b, s, ws, &P, &w)) return rc;
    if (int rc = check_run_args(dt, nsteps, step0, mode)) return rc;
    if ((mode & SPH_RUN_GRAPH) && !stream)
        return fail(SPH_E_INVAL, "SPH_RUN_GRAPH needs a stream other than NULL");
    if ((mode & SPH_RUN_LAGGED) && P.scheme != SPH_SCHEME_VERLET)
        return fail(SPH_E_INVAL, "SPH_RUN_LAGGED needs the Verlet scheme");
    return run_steps(P, *s, w, nsteps, dt, step0, mode, static_cast<hipStream_t>(stream));
}

int sph_batch_run_profiled(const sph_batch *b, sph_state *s, void *ws, int64_t nsteps, double dt,
                           int64_t step0, int32_t mode, int32_t region, void *const *ev_begin,
                           void *const *ev_end, void *stream) {
    Problem P;
    Ws w;
    if (int rc = validate_batch(b, s, ws, &P, &w)) return rc;
    if (int rc = check_run_args(dt, nsteps, step0, mode & ~SPH_RUN_GRAPH)) return rc;
    if (mode & SPH_RUN_GRAPH) return fail(SPH_E_INVAL, "profiled runs take no graph");
    if ((mode & SPH_RUN_LAGGED) && P.scheme != SPH_SCHEME_VERLET)
        return fail(SPH_E_INVAL, "SPH_RUN_LAGGED needs the Verlet scheme");
    if (int rc = check_events(nsteps, region, ev_begin, ev_end)) return rc;
    return run_steps(P, *s, w, nsteps, dt, step0, mode, static_cast<hipStream_t>(stream), region,
                     ev_begin, ev_end);
}

int sph_batch_diagnostics(const sph_batch *b, const sph_state *s, void *ws, sph_diag *out,
                          void *stream) {
    Problem P;
    Ws w;
    if (int rc = validate_batch(b, s, ws, &P, &w)) return rc;
    if (!out) return fail(SPH_E_INVAL, "out is NULL");
    if (!s->cells_valid) return fail(SPH_E_STATE, "diagnostics need current cells");
    return launch_diag(P, *s, w, nullptr, 0, out, nullptr, static_cast<hipStream_t>(stream));
}

}  // extern "C"
