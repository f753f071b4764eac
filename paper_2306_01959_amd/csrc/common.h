// Internal declarations shared by the HIP translation units of libwcsph.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "wcsph.h"

namespace wcsph {

constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kSortThreads = 256;    // radix sort workgroup
constexpr int kSortItems = 16;       // keys per thread per tile
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kChunk = 64;           // targets per interaction chunk (one wave)
constexpr int kDiagThreads = 256;
constexpr int kDiagBlocks = 512;     // fixed partial count: deterministic sums
constexpr int kDiagFields = 16;
constexpr int kMaxProbes = 1024;    // probe points per sph_diagnostics call

// Device-resident scalars inside the workspace.
struct DevScalars {
    unsigned long long dt_min_bits;  // bits of the running min of the dt bound
                                     // (positive doubles order like integers)
    double dt_cfl;                   // Cr * bound of the last interaction
    double dt_last;                  // dt used by the last step
    double time;                     // accumulated simulated time
    long long steps;                 // steps taken
    unsigned int nchunks;            // interaction chunks of the current cells
    unsigned int dt_cfl_violation;   // a step used dt > dt_cfl
    unsigned long long pairs[3];     // interacting pairs since init: FF, FB, BF
    unsigned int work;               // next interaction chunk to take
    unsigned int pad_;
};

// Byte offsets of the workspace regions (all 256-byte aligned).
struct WsLayout {
    int64_t n = 0;
    int64_t ncells = 0;
    int64_t nrows = 0;
    int64_t ntiles = 0;
    int64_t max_chunks = 0;
    int32_t key_bits = 0;
    int32_t precision = 0;
    size_t keys = 0, keys_alt = 0, vals = 0, vals_alt = 0;
    size_t sorted_keys = 0;  // keys or keys_alt, whichever holds the sort output
    size_t hist = 0;
    size_t cell_start = 0;
    size_t chunks = 0;
    size_t view0 = 0, view1 = 0, view2 = 0;
    size_t rates = 0;   // ax, ay, az, drho, mumax (each n values)
    size_t scalars = 0;
    size_t diag_part = 0;
    size_t total = 0;
    size_t view_elem = 0;  // bytes of one view record (per array)
    size_t rate_elem = 0;  // bytes of one rate value
};

WsLayout make_layout(const sph_params &p, int64_t n);

// Typed views into a workspace.
struct Ws {
    WsLayout L;
    char *base = nullptr;
    template <class T>
    T *at(size_t off) const { return reinterpret_cast<T *>(base + off); }
    uint32_t *keys() const { return at<uint32_t>(L.keys); }
    uint32_t *keys_alt() const { return at<uint32_t>(L.keys_alt); }
    uint32_t *vals() const { return at<uint32_t>(L.vals); }
    uint32_t *vals_alt() const { return at<uint32_t>(L.vals_alt); }
    uint32_t *hist() const { return at<uint32_t>(L.hist); }
    uint32_t *cell_start() const { return at<uint32_t>(L.cell_start); }
    int4 *chunks() const { return at<int4>(L.chunks); }
    DevScalars *scalars() const { return at<DevScalars>(L.scalars); }
    double *diag_part() const { return at<double>(L.diag_part); }
};

// Thread-local error reporting.
int fail(int code, const std::string &msg);
int hip_check(hipError_t e, const char *what);
int launch_check(const char *what);

// Grid and kernel constants shared by the kernels of one call.
struct Grid {
    double ox, oy, oz, cs, inv_cs;
    int nx, ny, nz;
};

inline Grid grid_of(const sph_params &p) {
    Grid g;
    g.ox = p.origin[0];
    g.oy = p.origin[1];
    g.oz = p.origin[2];
    g.cs = p.cell_size;
    g.inv_cs = 1.0 / p.cell_size;
    g.nx = p.dims[0];
    g.ny = p.dims[1];
    g.nz = p.dims[2];
    return g;
}

// Launchers implemented in the kernel translation units.
int launch_encode(const sph_params &p, const sph_state &s, const Ws &w, hipStream_t st);
int launch_sort(const Ws &w, hipStream_t st, uint32_t **sorted_keys, uint32_t **perm);
int launch_reorder(const sph_params &p, sph_state &s, const Ws &w, const uint32_t *keys,
                   const uint32_t *perm, hipStream_t st);
int launch_cell_table(const sph_params &p, const Ws &w, const uint32_t *keys, hipStream_t st);
int launch_chunks(const sph_params &p, const Ws &w, hipStream_t st);
int launch_interact(const sph_params &p, const sph_state &s, const Ws &w, hipStream_t st,
                    int32_t *st_nf = nullptr, int32_t *st_nb = nullptr,
                    uint32_t *st_hash = nullptr);
int launch_export_rates(const sph_params &p, const Ws &w, int64_t n, double *ax, double *ay,
                        double *az, double *drho, double *mumax, hipStream_t st);
int launch_integrate(const sph_params &p, sph_state &s, const Ws &w, double dt, int64_t step,
                     hipStream_t st);
int launch_diag(const sph_params &p, const sph_state &s, const Ws &w, const double *probes,
                int32_t np, sph_diag *out, double *probe_p, hipStream_t st);
int launch_set_density(const sph_params &p, sph_state &s, const double *rho, int which,
                       hipStream_t st);
int launch_get_density(const sph_params &p, const sph_state &s, double *rho, int which,
                       hipStream_t st);
int launch_ws_init(const Ws &w, hipStream_t st);
int set_split(int precision, int split);
int set_group(int precision, int group);
int split_for(const sph_params &p, int64_t max_chunks);
int group_for(const sph_params &p);

// Cell id layout: linear = cx + nx * (cy + ny * cz).
__host__ __device__ inline int64_t lin_cell(int cx, int cy, int cz, int nx, int ny) {
    return cx + (int64_t)nx * (cy + (int64_t)ny * cz);
}

}  // namespace wcsph
