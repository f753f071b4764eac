// extern "C" entry points of libwcsph: argument validation, workspace layout
// and the order of launches for each call.  Every argument is checked before
// anything is launched.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>

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

WsLayout make_layout(const sph_params &p, int64_t n) {
    WsLayout L;
    L.n = n;
    L.precision = p.precision;
    L.ncells = (int64_t)p.dims[0] * p.dims[1] * p.dims[2];
    L.nrows = (int64_t)p.dims[1] * p.dims[2];
    L.ntiles = (n + kSortTile - 1) / kSortTile;
    L.max_chunks = (n + kChunk - 1) / kChunk + L.nrows;
    int bits = 0;
    while (bits < 32 && ((int64_t)1 << bits) < L.ncells) ++bits;
    L.key_bits = bits;
    const int passes = bits <= 0 ? 1 : (bits + kRadixBits - 1) / kRadixBits;
    const bool mixed = p.precision == SPH_MIXED;
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
    L.vals = take(4 * (size_t)n);
    L.vals_alt = take(4 * (size_t)n);
    L.sorted_keys = (passes & 1) ? L.keys_alt : L.keys;
    L.hist = take(4 * (size_t)kRadix * (size_t)L.ntiles);
    L.cell_start = take(4 * (size_t)(L.ncells + 1));
    L.chunks = take(sizeof(int4) * (size_t)L.max_chunks);
    L.view0 = take(L.view_elem * (size_t)n);
    L.view1 = take(L.view_elem * (size_t)n);
    L.view2 = take((mixed ? 8 : 16) * (size_t)n);
    L.rates = take(5 * L.rate_elem * (size_t)n);
    L.scalars = take(sizeof(DevScalars));
    L.diag_part = take(sizeof(double) * ((size_t)kDiagBlocks * kDiagFields + kDiagFields +
                                         4 * (size_t)kMaxProbes));
    L.total = off;
    return L;
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
    if (nc >= ((int64_t)1 << 31) - 1) return fail(SPH_E_RANGE, "too many cells (>= 2^31)");
    if (p->precision != SPH_FP64 && p->precision != SPH_MIXED)
        return fail(SPH_E_INVAL, "unknown precision");
    if (p->c_mode != SPH_C_TAIT && p->c_mode != SPH_C_CONST)
        return fail(SPH_E_INVAL, "unknown c_mode");
    if (p->delta_pairs != SPH_DELTA_FLUID && p->delta_pairs != SPH_DELTA_ALL)
        return fail(SPH_E_INVAL, "unknown delta_pairs");
    if (p->reserved != 0) return fail(SPH_E_INVAL, "reserved must be 0");
    return SPH_OK;
}

static int check_n(int64_t n) {
    if (n < 1) return fail(SPH_E_INVAL, "n must be >= 1");
    if (n >= ((int64_t)1 << 31)) return fail(SPH_E_RANGE, "n must be < 2^31");
    return SPH_OK;
}

static bool aligned(const void *ptr, size_t a) { return ((uintptr_t)ptr % a) == 0; }

static int check_state(const sph_params *p, const sph_state *s) {
    if (!s) return fail(SPH_E_INVAL, "state is NULL");
    if (int rc = check_n(s->n)) return rc;
    const void *ptrs[] = {s->x,      s->y,      s->z,      s->ux,      s->uy,      s->uz,
                          s->uxm,    s->uym,    s->uzm,    s->rho,     s->rhom,    s->id,
                          s->x_alt,  s->y_alt,  s->z_alt,  s->ux_alt,  s->uy_alt,  s->uz_alt,
                          s->uxm_alt, s->uym_alt, s->uzm_alt, s->rho_alt, s->rhom_alt, s->id_alt};
    for (const void *q : ptrs) {
        if (!q) return fail(SPH_E_INVAL, "state array pointer is NULL");
        if (!aligned(q, 8) && !(p->precision == SPH_MIXED && aligned(q, 4)))
            return fail(SPH_E_INVAL, "state array pointer is misaligned");
    }
    const double *d8[] = {s->x, s->y, s->z, s->ux, s->uy, s->uz, s->uxm, s->uym, s->uzm,
                          s->x_alt, s->y_alt, s->z_alt, s->ux_alt, s->uy_alt, s->uz_alt,
                          s->uxm_alt, s->uym_alt, s->uzm_alt};
    for (const double *q : d8)
        if (!aligned(q, 8)) return fail(SPH_E_INVAL, "double array pointer is misaligned");
    if (p->precision == SPH_FP64) {
        const void *r8[] = {s->rho, s->rhom, s->rho_alt, s->rhom_alt};
        for (const void *q : r8)
            if (!aligned(q, 8)) return fail(SPH_E_INVAL, "density pointer is misaligned");
    }
    if (s->reserved != 0) return fail(SPH_E_INVAL, "state reserved must be 0");
    return SPH_OK;
}

static int check_ws(const sph_params *p, const sph_state *s, void *ws, Ws *out) {
    if (!ws) return fail(SPH_E_INVAL, "workspace is NULL");
    if (!aligned(ws, 256)) return fail(SPH_E_INVAL, "workspace must be 256-byte aligned");
    out->L = make_layout(*p, s->n);
    out->base = static_cast<char *>(ws);
    return SPH_OK;
}

static int validate(const sph_params *p, const sph_state *s, void *ws, Ws *w) {
    if (int rc = check_params(p)) return rc;
    if (int rc = check_state(p, s)) return rc;
    return check_ws(p, s, ws, w);
}

static int build_cells(const sph_params &p, sph_state &s, const Ws &w, hipStream_t st) {
    if (int rc = launch_encode(p, s, w, st)) return rc;
    uint32_t *keys = nullptr, *perm = nullptr;
    if (int rc = launch_sort(w, st, &keys, &perm)) return rc;
    if (int rc = launch_reorder(p, s, w, keys, perm, st)) return rc;
    if (int rc = launch_cell_table(p, w, keys, st)) return rc;
    if (int rc = launch_chunks(p, w, st)) return rc;
    s.cells_valid = 1;
    return SPH_OK;
}

static int one_step(const sph_params &p, sph_state &s, const Ws &w, double dt, int64_t step,
                    hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
    if (!s.cells_valid)
        if (int rc = build_cells(p, s, w, st)) return rc;
    if (ev0)
        if (int rc = hip_check(hipEventRecord(ev0, st), "event record")) return rc;
    if (int rc = launch_interact(p, s, w, st)) return rc;
    if (ev1)
        if (int rc = hip_check(hipEventRecord(ev1, st), "event record")) return rc;
    if (int rc = launch_integrate(p, s, w, dt, step, st)) return rc;
    s.cells_valid = 0;
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
    for (int k = 0; k < 4; ++k)
        if (t->reserved[k] != 0) return fail(SPH_E_INVAL, "tuning reserved must be 0");
    auto split_ok = [](int v) { return v == 0 || v == 1 || v == 3 || v == 9; };
    auto group_ok = [](int v) { return v == 0 || v == 8 || v == 16 || v == 64; };
    if (!split_ok(t->split_fp64) || !split_ok(t->split_mixed))
        return fail(SPH_E_INVAL, "split must be 0, 1, 3 or 9");
    if (!group_ok(t->group_fp64) || !group_ok(t->group_mixed))
        return fail(SPH_E_INVAL, "group must be 0, 8, 16 or 64");
    set_split(SPH_FP64, t->split_fp64);
    set_split(SPH_MIXED, t->split_mixed);
    set_group(SPH_FP64, t->group_fp64);
    set_group(SPH_MIXED, t->group_mixed);
    return SPH_OK;
}

int sph_get_split(const sph_params *p, int64_t n, int32_t *split, int32_t *group) {
    if (int rc = check_params(p)) return rc;
    if (int rc = check_n(n)) return rc;
    if (!split || !group) return fail(SPH_E_INVAL, "output is NULL");
    *split = split_for(*p, make_layout(*p, n).max_chunks);
    *group = group_for(*p);
    return SPH_OK;
}

int sph_workspace_bytes(const sph_params *p, int64_t n, size_t *bytes) {
    if (int rc = check_params(p)) return rc;
    if (int rc = check_n(n)) return rc;
    if (!bytes) return fail(SPH_E_INVAL, "bytes is NULL");
    *bytes = make_layout(*p, n).total;
    return SPH_OK;
}

int sph_workspace_init(const sph_params *p, int64_t n, void *ws, size_t ws_bytes, void *stream) {
    if (int rc = check_params(p)) return rc;
    if (int rc = check_n(n)) return rc;
    if (!ws) return fail(SPH_E_INVAL, "workspace is NULL");
    if (!aligned(ws, 256)) return fail(SPH_E_INVAL, "workspace must be 256-byte aligned");
    Ws w;
    w.L = make_layout(*p, n);
    w.base = static_cast<char *>(ws);
    if (ws_bytes < w.L.total) return fail(SPH_E_SIZE, "workspace too small");
    return launch_ws_init(w, static_cast<hipStream_t>(stream));
}

int sph_set_density(const sph_params *p, sph_state *s, const double *rho, int32_t which,
                    void *stream) {
    if (int rc = check_params(p)) return rc;
    if (int rc = check_state(p, s)) return rc;
    if (!rho || !aligned(rho, 8)) return fail(SPH_E_INVAL, "rho is NULL or misaligned");
    if (which != 0 && which != 1) return fail(SPH_E_INVAL, "which must be 0 or 1");
    return launch_set_density(*p, *s, rho, which, static_cast<hipStream_t>(stream));
}

int sph_get_density(const sph_params *p, const sph_state *s, double *rho, int32_t which,
                    void *stream) {
    if (int rc = check_params(p)) return rc;
    if (int rc = check_state(p, s)) return rc;
    if (!rho || !aligned(rho, 8)) return fail(SPH_E_INVAL, "rho is NULL or misaligned");
    if (which != 0 && which != 1) return fail(SPH_E_INVAL, "which must be 0 or 1");
    return launch_get_density(*p, *s, rho, which, static_cast<hipStream_t>(stream));
}

int sph_build_cells(const sph_params *p, sph_state *s, void *ws, void *stream) {
    Ws w;
    if (int rc = validate(p, s, ws, &w)) return rc;
    return build_cells(*p, *s, w, static_cast<hipStream_t>(stream));
}

int sph_interact(const sph_params *p, const sph_state *s, void *ws, double *ax, double *ay,
                 double *az, double *drho, double *mumax, void *stream) {
    Ws w;
    if (int rc = validate(p, s, ws, &w)) return rc;
    if (!ax || !ay || !az || !drho) return fail(SPH_E_INVAL, "output pointer is NULL");
    const double *outs[] = {ax, ay, az, drho};
    for (const double *q : outs)
        if (!aligned(q, 8)) return fail(SPH_E_INVAL, "output pointer is misaligned");
    if (mumax && !aligned(mumax, 8)) return fail(SPH_E_INVAL, "mumax is misaligned");
    if (!s->cells_valid) return fail(SPH_E_STATE, "sph_interact needs current cells (sph_build_cells)");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (int rc = launch_chunks(*p, w, st)) return rc;  // resets the dt bound
    if (int rc = launch_interact(*p, *s, w, st)) return rc;
    return launch_export_rates(*p, w, s->n, ax, ay, az, drho, mumax, st);
}

int sph_neighbour_stats(const sph_params *p, const sph_state *s, void *ws, int32_t *n_fluid_nbrs,
                        int32_t *n_boundary_nbrs, uint32_t *id_hash, void *stream) {
    Ws w;
    if (int rc = validate(p, s, ws, &w)) return rc;
    if (!n_fluid_nbrs || !n_boundary_nbrs || !id_hash)
        return fail(SPH_E_INVAL, "output pointer is NULL");
    if (!aligned(n_fluid_nbrs, 4) || !aligned(n_boundary_nbrs, 4) || !aligned(id_hash, 4))
        return fail(SPH_E_INVAL, "output pointer is misaligned");
    if (!s->cells_valid) return fail(SPH_E_STATE, "sph_neighbour_stats needs current cells");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (int rc = launch_chunks(*p, w, st)) return rc;
    return launch_interact(*p, *s, w, st, n_fluid_nbrs, n_boundary_nbrs, id_hash);
}

int sph_step(const sph_params *p, sph_state *s, void *ws, double dt, int64_t step_index,
             void *stream) {
    Ws w;
    if (int rc = validate(p, s, ws, &w)) return rc;
    if (!std::isfinite(dt)) return fail(SPH_E_INVAL, "dt must be finite");
    if (step_index < 0) return fail(SPH_E_INVAL, "step_index must be >= 0");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (s->cells_valid)
        if (int rc = launch_chunks(*p, w, st)) return rc;  // fresh dt bound
    return one_step(*p, *s, w, dt, step_index, st);
}

int sph_run(const sph_params *p, sph_state *s, void *ws, int64_t nsteps, double dt, int64_t step0,
            void *stream) {
    Ws w;
    if (int rc = validate(p, s, ws, &w)) return rc;
    if (!std::isfinite(dt)) return fail(SPH_E_INVAL, "dt must be finite");
    if (nsteps < 0 || step0 < 0) return fail(SPH_E_INVAL, "nsteps and step0 must be >= 0");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (nsteps > 0 && s->cells_valid)
        if (int rc = launch_chunks(*p, w, st)) return rc;
    for (int64_t k = 0; k < nsteps; ++k)
        if (int rc = one_step(*p, *s, w, dt, step0 + k, st)) return rc;
    return SPH_OK;
}

int sph_run_profiled(const sph_params *p, sph_state *s, void *ws, int64_t nsteps, double dt,
                     int64_t step0, void *const *ev_begin, void *const *ev_end, void *stream) {
    Ws w;
    if (int rc = validate(p, s, ws, &w)) return rc;
    if (!std::isfinite(dt)) return fail(SPH_E_INVAL, "dt must be finite");
    if (nsteps < 0 || step0 < 0) return fail(SPH_E_INVAL, "nsteps and step0 must be >= 0");
    if ((ev_begin == nullptr) != (ev_end == nullptr))
        return fail(SPH_E_INVAL, "ev_begin and ev_end must both be given or both be NULL");
    if (ev_begin)
        for (int64_t k = 0; k < nsteps; ++k)
            if ((ev_begin[k] == nullptr) != (ev_end[k] == nullptr))
                return fail(SPH_E_INVAL, "event handles of a step must both be set or both NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (nsteps > 0 && s->cells_valid)
        if (int rc = launch_chunks(*p, w, st)) return rc;
    for (int64_t k = 0; k < nsteps; ++k) {
        hipEvent_t e0 = ev_begin ? static_cast<hipEvent_t>(ev_begin[k]) : nullptr;
        hipEvent_t e1 = ev_end ? static_cast<hipEvent_t>(ev_end[k]) : nullptr;
        if (int rc = one_step(*p, *s, w, dt, step0 + k, st, e0, e1)) return rc;
    }
    return SPH_OK;
}

int sph_diagnostics(const sph_params *p, const sph_state *s, void *ws, const double *probes_xyz,
                    int32_t np, sph_diag *out, double *probe_p, void *stream) {
    Ws w;
    if (int rc = validate(p, s, ws, &w)) return rc;
    if (!out) return fail(SPH_E_INVAL, "out is NULL");
    if (np < 0 || np > kMaxProbes) return fail(SPH_E_INVAL, "np must be in [0, 1024]");
    if (np > 0 && (!probes_xyz || !probe_p)) return fail(SPH_E_INVAL, "probe arrays are NULL");
    if (!s->cells_valid) return fail(SPH_E_STATE, "sph_diagnostics needs current cells");
    return launch_diag(*p, *s, w, probes_xyz, np, out, probe_p, static_cast<hipStream_t>(stream));
}

}  // extern "C"
