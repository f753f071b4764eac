/*
 * wcsph.h -- C ABI of the MI355X (gfx950) WCSPH step library.
 *
 * The library advances a weakly-compressible SPH (WCSPH) particle system by
 * the step of Amaro Junior, Cheng & Buruchenko, "A comparison between
 * weakly-compressible SPH and moving particle semi-implicit methods for 3D
 * dam-break flows", Section 2.2:
 *   - neighbours: all j with |r_j - r_i| < 2h, j != i (compact support of
 *     the Wendland kernel, eq. sphw), found through a cell-linked list;
 *   - momentum (eq. sphu) with Tait pressure (eq. tait) and Monaghan
 *     artificial viscosity (eqs. pi, cpmu);
 *   - delta-SPH continuity (eq. sphrho);
 *   - Verlet update with an Euler reset every N_s steps (eqs. sphu1-sphrho1,
 *     sphu2-sphrho2), adaptive time step (eq. sphdt);
 *   - dynamic boundary particles: they obey continuity and the equation of
 *     state but are not moved by the forces (a wall stays put, a gate moves
 *     with its prescribed velocity).
 * Around that step, on the same cell list: a two-stage symplectic scheme
 * (sph_params.scheme), the loads of Section 3 (force on wall particles,
 * pressure impulse at probes), batches of independent systems, and the
 * explicit operators of the MPS method (Section 2).
 *
 * Conventions for every entry point:
 *   - extern "C"; the return value is an sph_status (0 = success).  On
 *     failure sph_last_error() returns a message for the calling thread.
 *     Arguments are validated before anything is launched; a rejected call
 *     launches nothing and changes nothing.
 *   - Device pointers are HIP device addresses (HBM) owned by the caller.  The
 *     library never allocates or frees device memory in these calls and holds
 *     no device state between calls; everything it needs lives in the caller's
 *     workspace buffer (size from sph_workspace_bytes, 256-byte aligned).
 *     The one exception is sph_run_noalloc, whose workspace is a static
 *     device array of the library.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls are
 *     asynchronous on that stream except those that return host values
 *     (sph_diagnostics, sph_batch_diagnostics, sph_boundary_force,
 *     sph_probe_impulse) and those whose description says they synchronise
 *     (sph_batch_workspace_init, sph_batch_run with SPH_RUN_GRAPH);
 *     sph_mps_constants runs on the host only.
 *   - Particle arrays are structure-of-arrays of length n.  After
 *     sph_build_cells the arrays are in cell order (per system: fluid
 *     before boundary, then cell row, then cell x); id[] carries each
 *     particle's original index.
 *   - One state/workspace pair must not be used by two overlapping calls.
 */
#ifndef WCSPH_H
#define WCSPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPH_ABI_VERSION 1

typedef enum {
    SPH_OK = 0,
    SPH_E_INVAL = -1,  /* bad argument: null/misaligned pointer, bad size or parameter */
    SPH_E_HIP = -2,    /* a HIP runtime call or kernel launch failed */
    SPH_E_RANGE = -3,  /* a size does not fit the 32-bit index space */
    SPH_E_STATE = -4,  /* call out of order (e.g. interact before build_cells) */
    SPH_E_SIZE = -5    /* workspace too small for (params, n) */
} sph_status;

/* Arithmetic of the pair interaction. */
typedef enum {
    SPH_FP64 = 0,  /* FP64 everywhere; density stored as double rho */
    SPH_MIXED = 1  /* FP32 pair arithmetic on (integer cell, FP32 offset)
                      positions; FP64 position/velocity accumulators; density
                      stored as float (rho - rho0) */
} sph_precision;

/* Sound speed c_i in the viscosity average (eq. pi, cpmu). */
typedef enum {
    SPH_C_TAIT = 0,  /* c_i = c0 (rho_i/rho0)^((gamma-1)/2), the Tait sound speed */
    SPH_C_CONST = 1  /* c_i = c0 */
} sph_c_mode;

/* Pairs that carry the delta-SPH diffusive term (eq. sphrho). */
typedef enum {
    SPH_DELTA_FLUID = 0,  /* fluid i with fluid j only */
    SPH_DELTA_ALL = 1     /* fluid i with every neighbour j */
} sph_delta_pairs;

/*
 * Time-integration scheme of sph_step / sph_run / sph_batch_run.
 * SPH_SCHEME_VERLET: the paper's Verlet scheme with the Euler reset every
 * N_s steps (eqs. sphu1-sphrho1, sphu2-sphrho2), one interaction per step.
 * SPH_SCHEME_SYMPLECTIC: a two-stage symplectic predictor-corrector
 * (position Verlet, which the paper cites among the alternatives without
 * writing it out), two interactions per step:
 *   rates at t:   r* = r + dt/2 u,  u* = u + dt/2 a,  rho* = rho + dt/2 drho
 *   rates at t*:  u' = u + dt a*,   r' = r* + dt/2 u', rho' = rho + dt drho*
 * with dt fixed by the first stage (the caller's dt, or eq. sphdt on the
 * rates at t); afterwards (um, rhom) hold the level at t.  In both schemes
 * boundary particles update rho and move with their own constant velocity
 * (zero for fixed walls; the prescribed velocity of a moving gate, as in the
 * paper's gate-release case).
 */
typedef enum {
    SPH_SCHEME_VERLET = 0,
    SPH_SCHEME_SYMPLECTIC = 1
} sph_scheme;

/*
 * Problem parameters (Section 2.2 and Section 3 of the paper).  All lengths in
 * metres, SI units.  Validation (SPH_E_INVAL): dp > 0, h > 0, rho0 > 0,
 * c0 > 0, gamma >= 1, alpha >= 0, 0 <= delta <= 1, eta2_coef >= 0,
 * 0 < cfl <= 1, mass > 0, cell_size >= 2h, dims[k] >= 1 and
 * dims[0]*dims[1]*dims[2] < 2^29 (SPH_E_RANGE), finite values, enums in range
 * (scheme included).
 */
typedef struct sph_params {
    double dp;         /* initial particle spacing l0 */
    double h;          /* smoothing length (h = k_SPH l0) */
    double rho0;       /* reference density */
    double c0;         /* artificial speed of sound */
    double gamma;      /* Tait polytropic index */
    double alpha;      /* artificial viscosity coefficient */
    double delta;      /* delta-SPH coefficient */
    double g[3];       /* body force per unit mass (gravity) */
    double eta2_coef;  /* eta^2 = eta2_coef * h^2 (the paper: 0.01) */
    double cfl;        /* Courant number Cr of eq. sphdt */
    double mass;       /* particle mass (fluid and boundary) */
    double origin[3];  /* lower corner of the cell grid */
    double cell_size;  /* cell edge, >= 2h (2h(1 + 2^-20) recommended) */
    int32_t dims[3];   /* cells per axis; positions outside are binned to the
                          nearest cell (never dropped) and counted */
    int32_t verlet_ns; /* Euler reset period N_s (40); <= 0: Euler only at step 0 */
    int32_t precision; /* sph_precision */
    int32_t c_mode;    /* sph_c_mode */
    int32_t delta_pairs; /* sph_delta_pairs */
    int32_t scheme;    /* sph_scheme (0: the paper's Verlet scheme) */
} sph_params;

/*
 * Particle state, structure of arrays of length n, all device pointers.
 * Two Verlet levels: (u, rho) at t and (um, rhom) at t - dt.
 * rho/rhom: double rho when precision == SPH_FP64; float (rho - rho0) when
 * SPH_MIXED (use sph_set_density / sph_get_density to convert).
 * id: original index in bits 0..30, bit 31 set for a boundary particle.
 * The *_alt arrays are second buffers of the same sizes: sph_build_cells
 * gathers the state into them in cell order and swaps the pointer pairs in
 * this struct, and sph_step swaps (u, um) and (rho, rhom); read the pointers
 * back after each call.
 */
typedef struct sph_state {
    int64_t n;
    double *x, *y, *z;
    double *ux, *uy, *uz;
    double *uxm, *uym, *uzm;
    void *rho, *rhom;
    uint32_t *id;
    double *x_alt, *y_alt, *z_alt;
    double *ux_alt, *uy_alt, *uz_alt;
    double *uxm_alt, *uym_alt, *uzm_alt;
    void *rho_alt, *rhom_alt;
    uint32_t *id_alt;
    int32_t cells_valid; /* set by sph_build_cells; cleared when positions change */
    int32_t reserved;
} sph_state;

/* Host-side results of sph_diagnostics, all FP64 (sums in a fixed order). */
typedef struct sph_diag {
    double mass;        /* sum of m over all particles */
    double mom[3];      /* sum of m u over fluid particles */
    double e_kin;       /* sum of m |u|^2 / 2 over fluid */
    double e_pot;       /* sum of -m g . r over fluid */
    double e_int;       /* sum of m e(rho), e = (B/rho0)[(rho/rho0)^(gamma-1)/(gamma-1)
                           + rho0/rho - gamma/(gamma-1)], B = rho0 c0^2/gamma */
    double umax;        /* max |u| over fluid */
    double x_front;     /* max x over fluid particles with a fluid neighbour
                           (-inf if none) */
    double dt_cfl;      /* time-step bound of eq. sphdt at the last interaction */
    double dt_last;     /* dt used by the last sph_step */
    double time;        /* accumulated simulated time of sph_step calls */
    int64_t n;          /* particles */
    int64_t n_fluid;    /* fluid particles */
    int64_t n_outside;  /* particles outside the grid (binned by clamping) */
    int64_t n_nonfinite;/* non-finite values in r, u, rho */
    int64_t steps;      /* steps taken since sph_workspace_init */
    int64_t pairs_ff;   /* interacting ordered pairs evaluated since
                           sph_workspace_init: fluid i with fluid j, */
    int64_t pairs_fb;   /* fluid i with boundary j (counted as pairs_bf: the
                           neighbour relation is symmetric, exactly in FP64,
                           up to pairs within one FP32 rounding of 2h in
                           mixed precision), */
    int64_t pairs_bf;   /* boundary i with fluid j */
    uint32_t flags;     /* SPH_FLAG_* */
    uint32_t reserved;
} sph_diag;

#define SPH_FLAG_NONFINITE 1u   /* n_nonfinite > 0 */
#define SPH_FLAG_OUTSIDE 2u     /* n_outside > 0 */
#define SPH_FLAG_DENSITY 4u     /* some |rho - rho0| / rho0 > 0.1 */
#define SPH_FLAG_DT_CFL 8u      /* dt_last exceeded dt_cfl */

/* Library ABI version (SPH_ABI_VERSION). */
int sph_version(void);

/* Message describing the last failure on the calling thread ("" if none). */
const char *sph_last_error(void);

/* Validate params (see sph_params) without touching the device. */
int sph_check_params(const sph_params *p);

/* Decomposition of the interaction kernel. */
typedef enum {
    SPH_KERNEL_AUTO = 0,
    SPH_KERNEL_ROWS = 1,   /* chunks of up to 64 targets of one half-row (the
                              fluid or the boundary particles of a cell row,
                              never across an empty cell); `split`
                              waves (1, 3 or 9) divide the 9 stencil rows; inside
                              a wave the targets form groups of `group` (8, 16
                              or 64), each culled on its own */
    SPH_KERNEL_GROUPS = 2, /* one independent wave per group of up to `group`
                              targets of one half-row (8, 16 or 64), streaming
                              and culling its own candidates; `split` unused */
    SPH_KERNEL_COOP = 3,   /* four groups of `group` targets (8 or 16; 64 acts
                              as 16) per workgroup, which loads and culls their
                              candidates once for all four; `split` unused */
    SPH_KERNEL_COOP2 = 4   /* SPH_KERNEL_COOP with the pairs in two phases: the
                              neighbour test first, then the pair terms over
                              each target's neighbours only */
} sph_kernel;

/*
 * Launch shape of the interaction (an autotuner sets it): the kernel, the
 * waves per chunk, the targets per group (a wave step evaluates `group`
 * targets against 64/`group` candidates) and the order in which workgroups
 * take chunks: xcd_run = 1 in chunk order, 8 or 32 so that each of the
 * chip's eight XCDs (which receive workgroups in turn) takes runs of that
 * many consecutive chunks, which share candidates in its L2.  0 = the
 * library's choice (xcd_run: 1).  full_gather = 1 turns off the fixed-wall
 * shortcut of sph_run / sph_batch_run: from the third step of a call, while
 * no boundary particle has moved with the workspace, the boundary particles
 * keep their sorted positions and the gather leaves them in place, copying
 * only their densities; both give the same results bit for bit.  Per
 * precision (full_gather: for both), process-wide, host-side: besides sph_run_noalloc's scratch this
 * is the library's only state outside the caller's buffers.  It changes
 * launch shapes only, never results beyond summation order; each field is
 * read and written atomically, so a launch on another thread sees either the
 * old or the new value of each field (set it before launching for a
 * consistent shape).
 */
typedef struct sph_tuning {
    int32_t split_fp64;
    int32_t split_mixed;
    int32_t group_fp64;
    int32_t group_mixed;
    int32_t kernel_fp64;  /* sph_kernel */
    int32_t kernel_mixed;
    int32_t xcd_run_fp64;  /* 0, 1, 8 or 32 */
    int32_t xcd_run_mixed;
    int32_t full_gather;   /* 0 or 1, see above */
} sph_tuning;

int sph_set_tuning(const sph_tuning *t);

/* The launch shape the library uses for (p, n), after sph_set_tuning. */
int sph_get_split(const sph_params *p, int64_t n, int32_t *split, int32_t *group,
                  int32_t *kernel);

/* Bytes of workspace needed for (p, n particles); 0 < n < 2^31. */
int sph_workspace_bytes(const sph_params *p, int64_t n, size_t *bytes);

/*
 * Prepare a fresh workspace: clears its device scalars (simulated time, step
 * counter, time-step bound).  Call once before the first use of a workspace;
 * calling it again restarts the clock.  SPH_E_SIZE if ws_bytes is too small.
 */
int sph_workspace_init(const sph_params *p, int64_t n, void *ws, size_t ws_bytes,
                       void *stream);

/*
 * Convert an FP64 density array (device, n values, in the state's current
 * order) into the state's density storage: which = 0 -> rho, 1 -> rhom.
 * sph_get_density does the reverse into an FP64 device array.
 */
int sph_set_density(const sph_params *p, sph_state *s, const double *rho, int32_t which,
                    void *stream);
int sph_get_density(const sph_params *p, const sph_state *s, double *rho, int32_t which,
                    void *stream);

/*
 * Cell-linked list (neighbour search set-up).  The neighbours of a particle
 * are the particles within the compact support 2h of the Wendland kernel
 * (eq. sphw, q <= 2; Section 2.2); with cells of edge >= 2h they all lie in
 * the 27 cells around its own.  Hashes every position to its
 * cell (clamped to the grid), sorts the particles stably by class (fluid
 * before boundary), then cell row (fixed y, z), then cell x, then half of
 * the cell along y, then half along x (fluid particles only; LSD radix sort
 * of 32-bit keys), gathers
 * every state array into that order (the *_alt buffers, then swaps the
 * pointers) and builds the cell table, the chunk list and the interaction
 * view (per-particle pressure, sound speed, 1/rho, and for SPH_MIXED the FP32
 * offset of each particle from its cell centre).  Stable: particles with the
 * same key keep their previous relative order, so the result is
 * deterministic.  Inside sph_run / sph_batch_run the steps between refreshes
 * (step indices that are not multiples of the graph period, else of 40) sort
 * on the cell alone, so the halves within a cell keep the order of the last
 * refresh; neighbour sets and results do not depend on that order beyond
 * rounding.
 */
int sph_build_cells(const sph_params *p, sph_state *s, void *ws, void *stream);

/*
 * Rates of change at the current state (eqs. sphu, pi, cpmu, sphw, sphrho,
 * tait):
 *   fluid i:    a_i = -sum_j m [(P_i+P_j)/(rho_i rho_j) + Pi_ij] grad_i W_ij + g
 *               drho_i = sum_j m (u_i - u_j).grad_i W_ij
 *                        + 2 delta h c0 sum_j (rho_j - rho_i) F_ij m / rho_j
 *   boundary i: drho_i = sum_{j fluid} m (u_i - u_j).grad_i W_ij, a_i = 0
 * with grad_i W_ij = F_ij (r_j - r_i).  mumax_i = max_j |mu_ij|.
 * Requires sph_build_cells since the positions last changed (SPH_E_STATE).
 * Outputs are FP64 device arrays of n values in the current (cell) order;
 * mumax may be NULL.
 */
int sph_interact(const sph_params *p, const sph_state *s, void *ws, double *ax, double *ay,
                 double *az, double *drho, double *mumax, void *stream);

/*
 * Neighbour statistics at the current state, as decided by the interaction's
 * own pair predicate (see sph_interact): per particle, the number of fluid
 * neighbours, the number of boundary neighbours (boundary particles count
 * fluid neighbours only), and the sum modulo 2^32 of H(id_j) over the
 * neighbour set, H being the 32-bit MurmurHash3 finaliser of the original
 * index.  The hash identifies the set independently of visit order (test and
 * accounting aid).  int32/uint32 device arrays of n values, current order.
 * Requires current cells (SPH_E_STATE).
 */
int sph_neighbour_stats(const sph_params *p, const sph_state *s, void *ws, int32_t *n_fluid_nbrs,
                        int32_t *n_boundary_nbrs, uint32_t *id_hash, void *stream);

/*
 * One time step of the method: (sph_build_cells if the cells are stale) ->
 * interaction -> time step -> Verlet update.  dt > 0: use it; dt <= 0: use
 * the bound of eq. sphdt computed on the device from this step's rates (no
 * host synchronisation).  step_index n selects the Euler reset
 * (n mod verlet_ns == 0, and n == 0) or the two-level Verlet update.  Fluid
 * particles update r, u, rho; boundary particles rho only.  Afterwards the
 * positions have moved and cells_valid is 0.
 */
int sph_step(const sph_params *p, sph_state *s, void *ws, double dt, int64_t step_index,
             void *stream);

/*
 * nsteps calls of sph_step with step indices step0 .. step0+nsteps-1 and the
 * same dt rule, with every launch enqueued back to back on the stream.
 */
int sph_run(const sph_params *p, sph_state *s, void *ws, int64_t nsteps, double dt,
            int64_t step0, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): sph_run
 * without a caller workspace.  The workspace is a static device array of
 * SPH_NOALLOC_WS_BYTES inside the library; every GPU the library runs on holds
 * its own copy until the process ends (its address is looked up once per
 * device, on the stream's device).  The call allocates and frees nothing.
 * Problems whose workspace (sph_workspace_bytes) exceeds the array are
 * rejected with SPH_E_SIZE before anything is launched.
 * Every call starts a fresh clock: simulated time, step and pair counters
 * restart (as after sph_workspace_init), and the cell list is rebuilt from the
 * positions (cells_valid is cleared).  Calls on one GPU share the array:
 * calls that overlap in time on the same GPU (other streams, other threads)
 * race and must not be made.  Results equal those of sph_run on a fresh
 * workspace.
 */
#define SPH_NOALLOC_WS_BYTES (32u << 20)
int sph_run_noalloc(const sph_params *p, sph_state *s, int64_t nsteps, double dt, int64_t step0,
                    void *stream);

/* Regions of a step that sph_run_profiled can bracket with events. */
typedef enum {
    SPH_REGION_INTERACT = 0, /* the interaction kernel */
    SPH_REGION_SORT = 1,     /* the cell keys and all passes of the radix sort */
    SPH_REGION_REORDER = 2,  /* the gather into cell order (+ interaction view) */
    SPH_REGION_STEP = 3      /* the whole step */
} sph_region;

/*
 * sph_run that also records caller-created hipEvent_t handles on the stream
 * immediately before (ev_begin[k]) and after (ev_end[k]) one region of step
 * k (sph_region), for timing that region alone.  Both arrays hold nsteps
 * entries (a step whose two entries are NULL records nothing), or both
 * arrays are NULL (then it is sph_run).  An event record drains the stream,
 * so sampling a few steps disturbs the run least.
 */
int sph_run_profiled(const sph_params *p, sph_state *s, void *ws, int64_t nsteps, double dt,
                     int64_t step0, int32_t region, void *const *ev_begin, void *const *ev_end,
                     void *stream);

/*
 * FP64 global diagnostics of the current state and Shepard-filtered probe
 * pressures (eq. sphpa): P_a = sum_b P_b W_ab / sum_b W_ab over fluid b with
 * |r_b - a| < 2h; 0 for a probe with no fluid in range.  probes_xyz: host
 * array of 3*np doubles (may be NULL when np == 0); probe_p: host array of np
 * doubles.  Requires current cells (call after sph_build_cells; sph_step
 * leaves them stale).  Synchronises the stream.
 */
int sph_diagnostics(const sph_params *p, const sph_state *s, void *ws, const double *probes_xyz,
                    int32_t np, sph_diag *out, double *probe_p, void *stream);

/*
 * Load on a solid (Section 3, the force on the block): the sum over the
 * boundary particles inside the box [box[0], box[1]] x [box[2], box[3]] x
 * [box[4], box[5]] of m a_i, a_i being the pressure and viscosity terms of the
 * momentum equation (eqs. sphu, pi, cpmu, tait) that i's fluid neighbours
 * exert on it, as for a fluid particle; the body force is not included and
 * boundary-boundary pairs do not act (the wall particles stay where they are;
 * their accelerations serve only to obtain the force).  Arithmetic in FP64
 * from the state arrays in both precisions (the mixed state's densities are
 * FP32 rho - rho0).  box: host array of 6 finite values with lo <= hi
 * (SPH_E_INVAL otherwise).  force: host array of 3 doubles (N); count: the
 * boundary particles in the box (may be NULL).  Requires current cells
 * (SPH_E_STATE); synchronises the stream; the sum has a fixed order.
 */
int sph_boundary_force(const sph_params *p, const sph_state *s, void *ws, const double *box,
                       double *force, int64_t *count, void *stream);

/*
 * Probe pressures (eq. sphpa, as sph_diagnostics) and their pressure
 * impulse I_p = integral of P dt (Section 3, Table 2), accumulated in the
 * workspace by the trapezoidal rule over the samples of successive calls,
 * with the simulated time the steps have accumulated (sph_diag.time).  The
 * first call after sph_workspace_init, and any call with reset = 1, starts
 * the integral at this sample (impulse 0), and so does a call with a
 * different number of probes.  Successive calls must pass the same probe
 * points.  probes_xyz: host, 3 np finite values, 1 <= np <= 1024;
 * probe_p, impulse: host arrays of np doubles (Pa, Pa s).  Requires current
 * cells; synchronises the stream.
 */
int sph_probe_impulse(const sph_params *p, const sph_state *s, void *ws, const double *probes_xyz,
                      int32_t np, int32_t reset, double *probe_p, double *impulse, void *stream);

/*
 * Explicit operators of the moving particle semi-implicit (MPS) method
 * (Section 2, MPS subsection) on the same cell list, for comparing the two
 * methods' operators on one particle set.  With r_ij = r_j - r_i and the
 * weight w_ij = r_e / |r_ij| - 1 for 0 < |r_ij| < r_e, else 0 (eq. mpsw;
 * coincident particles, where it is unbounded, are left out), over all
 * other particles j, fluid and boundary:
 *   pnd_i   = sum_j w_ij                                         (eq. mpspnd)
 *   grad_i  = (3 / n0) sum_j (phi_j - phi_i) r_ij w_ij / |r_ij|^2 (eq. mpsgrad)
 *   lap_i   = (6 / (lambda0 n0)) sum_j (phi_j - phi_i) w_ij       (eq. mpslap)
 *   sigma_i = |sum_j r_ij w_ij| / sum_j w_ij, 0 without neighbours (eq. mpssigmai2)
 *   surface_i = 1 if pnd_i < beta1 n0 and sigma_i > rho1 l0, else 0
 *               (the two criteria of the NPCD test, eqs. mpsni, mpsisgmai1)
 * The pressure Poisson solve of the method is not part of this library.
 */
typedef struct sph_mps {
    double re;       /* effective radius r_e = k_MPS l0 (the paper: 2.1 l0) */
    double n0;       /* particle number density of a full support */
    double lambda0;  /* correction parameter of the Laplacian (eq. mpslambda) */
    double beta1;    /* density criterion, in (0, 1] (the paper: 0.98) */
    double rho1;     /* centroid criterion in units of l0, >= 0 (the paper: 0.2) */
    double l0;       /* initial particle distance */
} sph_mps;

/* n0 and lambda0 (eqs. mpspnd, mpslambda) of the fully filled support on
 * the cubic lattice of spacing l0; 0 < re <= 64 l0 (SPH_E_INVAL). */
int sph_mps_constants(double l0, double re, double *n0, double *lambda0);

/*
 * The operators above at every particle of a single system, in the current
 * (cell) order.  The current cells (SPH_E_STATE if stale) must be at least
 * r_e wide: m->re <= p->cell_size (SPH_E_INVAL), e.g. cells built with
 * h = r_e / 2.  phi: device array of n doubles (may be NULL: then lap and
 * grad must be NULL too).  Outputs are device arrays, each may be NULL:
 * pnd, lap, sigma n doubles; grad 3 n doubles (x components, then y, then
 * z); surface n int32.  Asynchronous on the stream.
 */
int sph_mps_operators(const sph_params *p, const sph_state *s, void *ws, const sph_mps *m,
                      const double *phi, double *pnd, double *lap, double *grad, double *sigma,
                      int32_t *surface, void *stream);

/* ======================================================================
 * Batches: an ensemble of independent systems advanced together, as in the
 * paper's artificial-viscosity study (Section 4: several alpha values on one
 * dam break) and its resolution study (several l0).  Every instance has its
 * own sph_params (grid, dp, h, mass, alpha, c0, ...), its own time step and
 * clock; particles of different instances never interact.  One cell hash,
 * one sort, one reorder, one interaction launch and one update per step
 * serve all instances: each instance's cells follow the previous instance's
 * in one global numbering.
 *
 * Particles: one sph_state holds all of them.  Instance k owns the original
 * ids [o_k, o_k + counts[k]) with o_k = counts[0] + ... + counts[k-1]; the
 * particles may come in any order (id bits 0..30 name the instance, bit 31
 * marks boundary particles as for a single system).
 */
#define SPH_MAX_INSTANCES 4096

typedef struct sph_batch {
    int32_t ninst;             /* 1 .. SPH_MAX_INSTANCES */
    int32_t reserved;          /* must be 0 */
    const sph_params *params;  /* host array of ninst; one precision for all */
    const int64_t *counts;     /* host array of ninst particle counts (>= 1) */
} sph_batch;

/* Run modes (bit flags) of sph_batch_run. */
#define SPH_RUN_LAGGED 1 /* step n > 0 takes dt = Cr x the bound of step n-1
                            (eq. sphdt one step late; step 0 its own bound), so
                            the interaction kernel advances each particle as
                            soon as its sums are complete: one fused kernel
                            instead of interaction + update */
#define SPH_RUN_GRAPH 2  /* capture a period of steps (lcm of 4 and every
                            N_s, at most 400) from the call's third step in
                            a HIP graph and replay it; the stream must not
                            be NULL; the call then synchronises the stream
                            before it returns */

/* Workspace bytes of a batch; SPH_E_RANGE if the sum of particles reaches
 * 2^31 or the sum of cells 2^29. */
int sph_batch_workspace_bytes(const sph_batch *b, size_t *bytes);

/*
 * Prepare a batch workspace: uploads the instance table (so the host arrays
 * of b may be freed on return) and clears every instance's clock.  Every
 * later sph_batch_* call on this workspace must pass the same batch
 * description; it is re-validated host-side on every call.  Synchronises
 * the stream.
 */
int sph_batch_workspace_init(const sph_batch *b, void *ws, size_t ws_bytes, void *stream);

/* Density conversion of a batch (see sph_set_density): each particle uses
 * its instance's rho0.  Requires an initialised workspace. */
int sph_batch_set_density(const sph_batch *b, sph_state *s, void *ws, const double *rho,
                          int32_t which, void *stream);
int sph_batch_get_density(const sph_batch *b, const sph_state *s, void *ws, double *rho,
                          int32_t which, void *stream);

/* sph_build_cells / sph_interact for a whole batch (same outputs, all n). */
int sph_batch_build_cells(const sph_batch *b, sph_state *s, void *ws, void *stream);
int sph_batch_interact(const sph_batch *b, const sph_state *s, void *ws, double *ax, double *ay,
                       double *az, double *drho, double *mumax, void *stream);

/*
 * nsteps steps of every instance (step indices step0 ..), dt > 0 for all
 * instances or dt <= 0 for each instance's own bound (eq. sphdt).  mode = 0
 * gives exactly sph_run on every instance; SPH_RUN_LAGGED and SPH_RUN_GRAPH
 * as above.  With SPH_RUN_LAGGED a step n > 0 needs the bound of an earlier
 * interaction on this workspace: without one that step takes dt = 0 and
 * raises SPH_FLAG_DT_CFL.
 */
int sph_batch_run(const sph_batch *b, sph_state *s, void *ws, int64_t nsteps, double dt,
                  int64_t step0, int32_t mode, void *stream);

/* sph_batch_run (no SPH_RUN_GRAPH) with events around one region, as
 * sph_run_profiled. */
int sph_batch_run_profiled(const sph_batch *b, sph_state *s, void *ws, int64_t nsteps, double dt,
                           int64_t step0, int32_t mode, int32_t region, void *const *ev_begin,
                           void *const *ev_end, void *stream);

/*
 * Per-instance diagnostics (see sph_diagnostics, without probes): out holds
 * ninst results.  Sums run over each instance's own particles; steps, the
 * pair counters and the CFL flag are totals of the batch.  Requires current
 * cells; synchronises the stream.
 */
int sph_batch_diagnostics(const sph_batch *b, const sph_state *s, void *ws, sph_diag *out,
                          void *stream);

#ifdef __cplusplus
}
#endif

#endif /* WCSPH_H */
