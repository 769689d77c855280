/*
 * moc.h - C ABI of the MI355X fixed-source 3D method-of-characteristics
 * transport library (gfx950, HIP).
 *
 * The library computes the per-iteration transport sweep of 3D MOC
 * (paper section 2.1, Eqs. 1-4) over 3D characteristic tracks generated on the
 * fly from stored 2D radial tracks and axial z-stacks (section 2.2, Eqs. 5-11;
 * section 3.2, Eq. 13), inside fixed-source source iteration:
 *
 *   geometry + track parameters + multigroup cross sections + fixed source
 *     -> converged FSR scalar flux.
 *
 * Conventions shared by every entry point
 *  - Every function returns MOC_OK (0) or a negative moc_status and never
 *    throws.  The text of the last error of the calling thread is returned by
 *    moc_last_error(); it stays valid until that thread's next call.
 *  - Host arrays passed in are read during the call only (copied); the caller
 *    keeps ownership and may free them on return.
 *  - Device memory is never allocated in the solve path: the caller passes a
 *    device workspace of at least moc_plan_info.workspace_bytes bytes (any
 *    device allocation, e.g. a torch uint8 tensor) and keeps it alive while
 *    the solver exists.  The stream is caller-owned (a hipStream_t passed as
 *    void*; NULL = the default stream).  All device work of a solver is issued
 *    on that stream; calls that return host data synchronise it.
 *  - Numbering contract:
 *      cell     = cy*nx + cx
 *      local    = 2*sector + (inside ? 0 : 1)   when inclusion_radius > 0
 *               = sector                        otherwise
 *      sector   = floor(atan2(y-yc, x-xc) mod 2pi / (2pi/n_sectors) + 1e-9)
 *                 mod n_sectors  (points on a sector line join the sector
 *                 that starts there)
 *      region r = cell*regions_per_cell + local
 *      FSR j    = r*n_layers + k,   k = floor(z / (height/n_layers))
 *    Fluxes and sources are [n_fsr][n_groups] row-major doubles.
 *  - 3D segments shorter than 1e-9 cm are dropped; a z-stack line is a 3D
 *    track only if it runs more than 1e-9 cm (2D length) inside the box, and a
 *    track leaving within 1e-9 cm of a box edge reflects across both faces.
 *  - Directed 3D tracks: stored tracks are numbered in z-stack order
 *    (Eq. 13: stored azimuth, 2D track within azimuth, polar angle, position
 *    in the stack); each is swept forward (dir 0) and backward (dir 1).
 */
#ifndef MOC_H
#define MOC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MOC_API __attribute__((visibility("default")))

typedef enum {
    MOC_OK = 0,
    MOC_EINVAL = -1,    /* invalid argument: bad geometry, tracking, XS, source, size */
    MOC_ENOMEM = -2,    /* workspace / budget smaller than required                  */
    MOC_EDEVICE = -3,   /* a HIP runtime error; moc_last_error() carries its text    */
    MOC_ENOTCONV = -4,  /* max_iters reached before tol; the flux is still valid     */
    MOC_EBUSY = -5      /* serving: request not finished yet                         */
} moc_status;

enum { MOC_BC_VACUUM = 0, MOC_BC_REFLECTIVE = 1 };
enum { MOC_FACE_XMIN = 0, MOC_FACE_XMAX, MOC_FACE_YMIN, MOC_FACE_YMAX, MOC_FACE_ZMIN, MOC_FACE_ZMAX };

/* Axially extruded pin-cell lattice (paper section 2.2: radial geometry
 * identical on every axial plane, materials per radial region).
 * Box [0, nx*pitch] x [0, ny*pitch] x [0, height], n_layers equal layers. */
typedef struct {
    int nx, ny;
    double pitch;
    double inclusion_radius;   /* 0: plain square cell; else < pitch/2            */
    int n_sectors;             /* 1, 2, 4, 8 or 16 equal sectors starting at +x   */
    double height;
    int n_layers;
    int bc[6];                 /* per face, MOC_BC_* (x-, x+, y-, y+, z-, z+)     */
    const int *cell_material;  /* [ny*nx][2] = {inside, outside} material ids     */
} moc_geometry;

/* Track laydown: n_azim azimuthal angles over [0, 2pi) (multiple of 4),
 * n_polar Gauss-Legendre polar angles over (0, pi) (even), radial track
 * spacing and axial ray spacing (Eq. 5's delta z) in cm.  Both are adjusted
 * down to the nearest cyclic values. */
typedef struct {
    int n_azim, n_polar;
    double radial_spacing, axial_spacing;
} moc_tracking;

/* Multigroup cross sections, isotropic scattering.
 * sigma_t [M][G] > 0, sigma_s [M][G][G] >= 0 indexed [m][g_from][g_to],
 * with sum_{g_to} sigma_s[m][g][g_to] < sigma_t[m][g] (source iteration
 * then contracts).  1 <= G <= 64. */
typedef struct {
    int n_groups, n_materials;
    const double *sigma_t;
    const double *sigma_s;
} moc_xs;

typedef struct moc_plan moc_plan;
typedef struct moc_solver moc_solver;
typedef struct moc_server moc_server;

typedef struct {
    long long n_fsr, n_regions;
    long long n_2d_tracks, n_2d_segments;
    long long n_stacks;        /* n_2d_tracks * n_polar                           */
    long long n_3d_tracks;     /* stored 3D tracks (each swept in 2 directions)   */
    long long n_chunks;        /* bundles of tracks_per_wave consecutive stack lines */
    int n_groups, tracks_per_wave;
    double dz;                 /* effective axial ray spacing                      */
    size_t workspace_bytes;    /* device bytes moc_solver_create needs             */
    size_t psi_bytes;          /* of which: the two boundary angular-flux buffers  */
    size_t workspace_bytes_fp64; /* bytes for FP64 boundary flux (needed by the    */
                                 /* FP64 sweep to keep full precision)             */
    int line_stride;           /* most lines between neighbouring lanes of a sweep */
                               /* bundle (lines per axial layer)                  */
    size_t workspace_bytes_chain; /* bytes for a chain-only solver: no boundary    */
                                  /* buffers (moc_solver_set_chain; 0: the plan has */
                                  /* no vacuum top and bottom faces)                */
    long long n_chain_segments;   /* independent jobs of a chain-line sweep        */
    long long n_chain_items;      /* units they sweep, in all (moc_plan_chain)     */
} moc_plan_info;

/* Solve controls.  sweep_fp64 = 1 runs segment arithmetic and angular flux in
 * FP64 (precision study); exp_mode 0 = stable 1 - e^-tau (polynomial below
 * tau = ln(2)/2, hardware exp2 above; within 4 ulp), 1 = the naive 1 - exp(-tau)
 * with the hardware exponential (precision study only). */
typedef struct {
    double tol;                /* stop when the L-inf relative flux change < tol  */
    int max_iters;
    int sweep_fp64;
    int exp_mode;
} moc_solve_opts;

typedef struct {
    int iters;
    double residual;           /* max_{j,g} |phi_k - phi_{k-1}| / phi_k            */
    double balance_lhs;        /* sum_{j,g} sum_s W dpsi of the last sweep (FP64)  */
    double balance_rhs;        /* sum W psi_in(k-1) - sum W psi_out(k), last sweep */
    double absorption, leakage, source;  /* physical totals at the last iterate   */
    unsigned long long seg_group_updates; /* per sweep: directed 3D segments x G  */
    unsigned long long link_errors;       /* exits whose successor was not found  */
    double sweep_ms_median;    /* median sweep-kernel time over the iterations    */
                               /* (moc_solve with graph-captured iterations: the  */
                               /* median time of a whole captured iteration)      */
} moc_stats;

/* ---------------------------------------------------------------- plan */

/* Host-side planning (paper section 3.1: geometry and 2D ray tracing on the
 * CPU): quadrature, cyclic 2D laydown, 2D ray tracing of the radial geometry,
 * reflective cycles and chain phases, z-stack table (Eq. 13) and the device
 * footprint.  Returns MOC_EINVAL for: n_azim not a positive multiple of 4;
 * n_polar odd or < 2; spacing <= 0; radius < 0 or >= pitch/2; n_sectors not
 * in {1,2,4,8,16}; G outside [1,64]; sigma_t <= 0; sigma_s < 0; out-scatter
 * ratio >= 1; material id out of range; bc not 0/1. */
MOC_API int moc_plan_create(const moc_geometry *geom, const moc_tracking *trk, const moc_xs *xs,
                            moc_plan **out);
/* Sizes of the plan and the device footprint of the data that section 3.1
 * copies to the GPU for 3D tracing and the sweep (the admission key of the
 * serving calls).  EINVAL on NULL. */
MOC_API int moc_plan_query(const moc_plan *plan, moc_plan_info *out);
/* Frees the host plan (lifetime only; no step of the method).  NULL-safe. */
MOC_API void moc_plan_destroy(moc_plan *plan);

/* Planner introspection (host, no device needed) of the quantities the paper
 * defines and this library stores: the angular quadrature indexed by azimuth
 * m and polar angle n (section 2.1, Eq. 2), the 2D tracks of section 3.1's
 * CPU ray tracing, the z-stacks of Eq. 5 (section 2.2) laid out as the
 * Z-STACK table of Eq. 13 (section 3.2), and the 2D segments.  Sizes follow
 * moc_plan_info; any pointer may be NULL to skip that output; EINVAL for a
 * NULL plan or a chunk out of range.
 *  quadrature: phi [n_azim/2] corrected azimuths, dphi [n_azim/2] azimuthal
 *    weights, spacing [n_azim/2] corrected radial spacing, cot [n_azim/2][n_polar]
 *    corrected polar cotangents, weight [n_azim/2][n_polar] track weights
 *    (solid angle x perpendicular area).
 *  tracks2d: xy [n][4] start/end points, length [n], azim [n],
 *    link [n][2] directed successor ids (2*t+d) of (t,fwd) and (t,bwd),
 *    chain [n] chain coordinate of the start point, sigma [n] +1/-1.
 *  stacks: zeta [n_stacks] phase of Eq. 5 in [0,dz), i_lo [n_stacks] index of
 *    the lowest line, count [n_stacks] lines in the stack (3D tracks).
 *  segments2d: pos [n_2d_segments] start position along its 2D track,
 *    region [n_2d_segments], first [n_2d_tracks+1] offsets per 2D track. */
MOC_API int moc_plan_quadrature(const moc_plan *plan, double *phi, double *dphi, double *spacing,
                                double *cot, double *weight);
MOC_API int moc_plan_tracks2d(const moc_plan *plan, double *xy, double *length, int *azim,
                              long long *link, double *chain, int *sigma);
MOC_API int moc_plan_stacks(const moc_plan *plan, double *zeta, long long *i_lo, long long *count);
MOC_API int moc_plan_segments2d(const moc_plan *plan, double *pos, int *region, long long *first);
/* Chain-line sweep segments (moc_solver_set_chain): first [n_chain_segments+1]
 * item offsets; per segment k [n] (its index in its directed cycle), nk [n]
 * (segments of that cycle) and lc [n] (the cycle's length); per item
 * code [n_chain_items] (unit 2*t + dir) and u [n_chain_items] (the unit's
 * start unrolled along the cycle).  Any pointer may be NULL. */
MOC_API int moc_plan_chain(const moc_plan *plan, long long *first, int *k, int *nk, double *lc,
                           int *code, double *u);
/* Chunks: work item w = 2*chunk + dir covers stored tracks
 * [first_track, first_track + n_tracks) swept in direction dir. */
MOC_API int moc_plan_chunk(const moc_plan *plan, long long chunk, long long *first_track,
                           int *n_tracks);

/* ---------------------------------------------------------------- solver */

/* Bind a plan to a caller-owned device workspace and stream; uploads the plan
 * (2D segments, z-stack table, links, cross sections: the data section 3.1
 * moves to the GPU) and computes the track-estimated FSR volumes V_j of the
 * Eq. 4 estimator with one volume sweep.  With ws_bytes >=
 * workspace_bytes_fp64 the boundary angular flux is stored in FP64, with
 * ws_bytes >= workspace_bytes in FP32.  A workspace of at least
 * workspace_bytes_chain (when that is nonzero) but less than workspace_bytes
 * makes a chain-only solver: it holds no boundary buffers, sweeps in chain
 * mode (moc_solver_set_chain) and refuses to leave it, as well as
 * moc_sweep_items and moc_get_boundary_flux.  ENOMEM below that.  The plan may
 * be destroyed afterwards. */
MOC_API int moc_solver_create(const moc_plan *plan, void *dev_workspace, size_t ws_bytes,
                              void *stream, moc_solver **out);
/* Lifetime only: NULL-safe; does not free the caller's workspace. */
MOC_API void moc_solver_destroy(moc_solver *s);

/* Fixed volumetric isotropic source Q of Eq. 1 (section 2.1), per FSR and
 * group: q [n_fsr][G] (finite, >= 0), copied to the device.  EINVAL for a
 * wrong size or a negative / non-finite value. */
MOC_API int moc_set_source(moc_solver *s, const double *q, size_t n);

/* Source iteration (section 2.1: Eq. 3 along every characteristic of both
 * directions, Eq. 4 scalar-flux estimate, repeated with the updated
 * scattering source until the flux stops changing) from phi = 0, psi = 0
 * until the residual max |phi_k - phi_{k-1}| / phi_k < tol or max_iters.
 * Each iteration is three launches (source update, on-the-fly sweep of
 * section 2.2 Eqs. 5-11, finalize); the host reads 8 bytes per iteration.
 * Returns MOC_OK, or MOC_ENOTCONV when max_iters was reached (flux valid);
 * EINVAL for bad options. */
MOC_API int moc_solve(moc_solver *s, const moc_solve_opts *opts, moc_stats *stats);

/* How the FP32 sweep generates the 3D segments of section 2.2 (Eqs. 6-11,
 * evaluated per line) for lines whose groups sit in one lane (G <= 8):
 * 1 = lockstep (every lane of a wave takes each 2D segment together),
 * 2 = per-lane (each lane takes one piece of its own line per step and moves
 * on to its next 2D segment by itself), 0 = automatic (per-lane for G <= 8, the
 * default).  Both walks give every line the same pieces in the same order:
 * results differ only by the order of FP64 additions.  The batched serving
 * sweep always takes the per-lane walk.  moc_solver_walk reports the walk in
 * use (1 or 2). */
MOC_API int moc_solver_set_walk(moc_solver *s, int walk);
/* Workgroup size of the per-lane sweep and the window of 2D segments its LDS
 * holds (the tally and reduced source of every layer and group of the
 * window's segments, section 2.1 Eqs. 3-4): 0 = automatic (256 threads with
 * 40 KB windows on shallow stacks, 1024 threads with up to 156 KB windows on
 * deep ones, else 512 threads with 64-78 KB), or 256, 512, 1024 to force one.
 * EINVAL for other values or when no window of that size fits.  Drops any
 * segment store.  moc_solver_window reports the size and the segments per
 * window in use. */
MOC_API int moc_solver_set_window(moc_solver *s, int threads);
MOC_API int moc_solver_window(const moc_solver *s, int *threads, int *segments);
MOC_API int moc_solver_walk(const moc_solver *s, int *walk);

/* Stored-segment sweep (the paper's EXP method with its memory management,
 * section 4.2): the 3D pieces of the units (2D track, direction) with the
 * largest footprint are generated once and kept in the caller's device
 * buffer dev_store (store_bytes, 256-byte aligned; caller-owned, kept alive
 * while the solver uses it), taken in decreasing footprint while they fit;
 * later FP32 per-lane sweeps replay them with a transport-only kernel and
 * sweep the remaining units on the fly, in that order on the solver's stream.
 * Results equal those of the on-the-fly sweep up to the order of FP64
 * additions.  The store serves the FP32 per-lane sweep only (G <= 8); the
 * FP64 sweep, the lockstep walk and the test hooks sweep on the fly.
 * dev_store = NULL or store_bytes = 0 drops the store.  info (optional)
 * reports what was stored and, once the units were counted (a buffer of at
 * least 20 bytes per unit), the buffer size that would hold them all.  EINVAL when the per-lane sweep does not apply.
 * Changing the schedule drops the store. */
typedef struct {
    long long units_stored, units_total;
    unsigned long long wave_steps_stored, wave_steps_total;  /* 64-lane steps of the walk */
    size_t bytes_used;
    size_t bytes_all;          /* buffer that would hold every unit (0 if not counted) */
} moc_store_info;
MOC_API int moc_solver_store_segments(moc_solver *s, void *dev_store, size_t store_bytes,
                                      moc_store_info *info);

/* Schedule of the work units (load balancing, paper section 4.3).  order:
 * 0 = decreasing work (lines x 2D segments; the default), 1 = natural (2D
 * track order of Eq. 13), 2 = decreasing work in groups of the resident
 * workgroup count with every other group reversed (the paper's alternating
 * sort).  persistent: 0 = one workgroup per unit, dispatched in list order;
 * 1 = a grid of the resident workgroup count, workgroup b sweeping units
 * b, b + grid, ... (a static assignment, like a grid-stride loop over
 * tracks; with FP32 boundary storage only, else one workgroup per unit).
 * Applies to the FP32 per-lane sweep; drops any store.  EINVAL for other
 * values. */
MOC_API int moc_solver_set_schedule(moc_solver *s, int order, int persistent);

/* Within one work unit (section 4.3's load balancing, inside a workgroup):
 * how the waves of a workgroup share the 64-line bundles of a window.
 * mode 0 = static (wave w takes bundles w, w + waves, ...); 1 = dynamic (a
 * wave that finishes a bundle takes the next one not yet taken); -1 =
 * automatic (dynamic from an estimated 4 bundles per wave in the window,
 * static below; the default).  Only which wave sweeps which lines changes, so results agree
 * up to the order of the FP64 tally additions.  EINVAL for other values. */
MOC_API int moc_solver_set_bundles(moc_solver *s, int mode);

/* Chain-line sweeping (section 2.1: Eqs. 2-4 solved along whole
 * characteristic lines; section 2.2: the z-stack lines of Eq. 5 continued
 * across the reflective side faces).  on = 1: each sweep follows every line
 * from the z face it enters through to the one it leaves through, the flux
 * leaving a track through a side face entering the reflected track within
 * the same sweep, instead of one sweep later through the boundary buffers
 * (the default, on = 0).  The fixed point is the same; the iterates differ
 * (no lag).  Each directed 2D cycle is cut into segments of lines by where
 * they enter the box (moc_plan_info.n_chain_segments in all); workgroups
 * take segments in turn and sweep their units in cycle order, passing the
 * flux in per-workgroup carry buffers.  Needs vacuum top and bottom faces,
 * an even polar count and the per-lane FP32 sweep (at most 8 groups);
 * EINVAL otherwise, and moc_solve / moc_iterate / moc_solve_eigen return
 * EINVAL in chain mode with options that select another sweep (FP64 or the
 * naive exponential).  Drops captured steps. */
MOC_API int moc_solver_set_chain(moc_solver *s, int on);

/* Eigenvalue mode: power iteration on k-eff (the multiplication factor the
 * paper's validation reports, Table 2).  nu_sigma_f and chi are [M][G]
 * (M = the plan's materials; finite, >= 0, nu_sigma_f not all zero), copied
 * to the device.  From phi = 1, psi = 0, k = 1, every iteration puts
 * chi_g F_j / k with F_j = sum_g nu_sigma_f phi_j,g in place of the fixed
 * source (which it overwrites: call moc_set_source again before a
 * fixed-source solve), runs one source iteration (source update, sweep,
 * finalize), sets k <- k P_new / P_old with P = sum_j V_j F_j, and takes as
 * residual the larger of |dk| / k and the largest change of the normalised
 * fission source over fissile FSRs (1 at the first iteration).  Stops when
 * the residual < tol after the first iteration (MOC_OK) or at max_iters
 * (MOC_ENOTCONV; flux and k valid).  *k_eff receives k; the flux (not
 * normalised) is read with moc_get_flux.  opts->sweep_fp64 selects the FP64
 * sweep; EINVAL for bad data or when no FSR produces fission neutrons. */
MOC_API int moc_solve_eigen(moc_solver *s, const double *nu_sigma_f, const double *chi,
                            const moc_solve_opts *opts, double *k_eff, moc_stats *stats);

/* Restart the source iteration of section 2.1 (phi = 0, boundary psi = 0,
 * iteration counter 0). */
MOC_API int moc_reset(moc_solver *s);
/* Run n further source iterations (section 2.1, Eqs. 3-4; source update,
 * sweep, finalize) without a host synchronisation between them; stats
 * (optional) synchronises once.  EINVAL for n < 1 or bad options. */
MOC_API int moc_iterate(moc_solver *s, int n, const moc_solve_opts *opts, moc_stats *stats);

/* The scalar flux of the last iterate (Eq. 4, section 2.1), host_out
 * [n_fsr][G] FP64; n must be n_fsr * G (EINVAL otherwise).  Synchronises. */
MOC_API int moc_get_flux(const moc_solver *s, double *host_out, size_t n);
/* The track-estimated FSR volumes V_j of Eq. 4, host_out [n_fsr].  Synchronises. */
MOC_API int moc_get_volumes(const moc_solver *s, double *host_out, size_t n);
/* Device address of the Eq. 4 scalar flux [n_fsr][G] FP64 inside the
 * workspace (valid while the solver exists; no copy). */
MOC_API int moc_flux_device_ptr(const moc_solver *s, const double **dev);

/* Test hook: the Eq. 3 sweep (section 2.1) of the listed work items
 * (2*chunk + dir) only, with the kernels and launch layout of the full sweep
 * restricted to them, from a
 * given reduced source qhat [n_fsr][G] (rounded to the sweep precision) and
 * incoming angular flux psi_in [n_items][tracks_per_wave][G] (lines beyond a
 * chunk's count are ignored).  Returns the FSR tallies acc [n_fsr][G]
 * (sum of W * delta_psi of those tracks) and every track's outgoing flux
 * psi_out [n_items][tracks_per_wave][G]. */
MOC_API int moc_sweep_items(moc_solver *s, long long n_items, const long long *items,
                            const double *qhat, const double *psi_in, int sweep_fp64,
                            double *acc_out, double *psi_out);

/* Test hook: the reduced source qhat = (sum_g' Sigma_s phi + Q) / (4 pi Sigma_t)
 * (the flat-source term of Eq. 3) of the solver's last source update, as the
 * sweep read it: fp64 = 0 gives the FP32 values of the FP32 sweep (widened),
 * 1 the FP64 values.  host_out [n_fsr][G]; n must be n_fsr * G.
 * Synchronises the stream. */
MOC_API int moc_get_reduced_source(const moc_solver *s, int fp64, double *host_out, size_t n);

/* Test hook: the incoming angular flux that the next source iteration's sweep
 * reads for the directed 3D tracks slots[i] = 2 * stored track + dir (the
 * boundary exchange of section 2.1's characteristic sweep, lagged one
 * iteration).  out [n][G], widened from the storage precision.  Only tracks
 * that enter through a reflective face carry a flux; the entries of tracks
 * entering through a vacuum face are stale and are not read by the sweep.
 * EINVAL for a slot outside [0, 2 * n_3d_tracks).  Synchronises the stream. */
MOC_API int moc_get_boundary_flux(const moc_solver *s, long long n, const long long *slots,
                                  double *out);

/* Test hook: the 3D segments (section 2.2, Eqs. 5-11) the GPU generates on
 * the fly for stored tracks
 * track_ids [n] (forward order): FSR ids and lengths written at
 * [i*cap, i*cap + count[i]) of fsr_out / len_out (count may exceed cap, then
 * only cap are written). */
MOC_API int moc_trace_tracks(moc_solver *s, long long n, const long long *track_ids, int cap,
                             int *fsr_out, double *len_out, int *count_out);

/* Test hook: the sweep's FP32 attenuation factor F(tau) = 1 - exp(-tau) of
 * Eq. 3, evaluated on the device by the same device function the sweep uses
 * (exp_mode 0: stable form; 1: naive 1 - exp) for n host values tau >= 0;
 * FP32 results to the host array out [n].  Allocates and frees its own
 * device buffers (not part of the solve path); synchronous. */
MOC_API int moc_eval_attenuation(const float *tau, long long n, int exp_mode, float *out);

/* The same evaluation for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): no device allocation and no free.  tau and out are host arrays
 * as above; the values are staged through a fixed array of 2^20 inputs and
 * 2^20 outputs that each device holds from the first call on it until the
 * process ends.  EINVAL for n > 2^20 (nothing is evaluated).  Synchronous on
 * the calling thread's current device; calls that overlap on one device
 * (from several threads) share that array and race. */
MOC_API int moc_eval_attenuation_noalloc(const float *tau, long long n, int exp_mode, float *out);

/* ---------------------------------------------------------------- serving */

/* Continuous batching of independent fixed-source solves on one GPU (the
 * paper's track-level parallelism, section 4.1, applied across requests).
 * The caller passes a device arena (256-byte aligned, caller-owned, kept
 * alive until destroy); the server carves its tables from the front and
 * sub-allocates one workspace per admitted request from the rest (first
 * fit).  At most max_slots requests run at once.  stream: a non-default
 * stream enables HIP-graph capture of the batched step (NULL: plain
 * launches).  Calls from one thread at a time. */
MOC_API int moc_server_create(void *dev_arena, size_t arena_bytes, int max_slots, void *stream,
                              moc_server **out);
/* Lifetime only: NULL-safe; waits for the stream; the arena stays the caller's. */
MOC_API void moc_server_destroy(moc_server *srv);
/* Bytes of the arena the server keeps for its own tables (host-only query):
 * a request fits when its workspace_bytes fits in the rest.  Serving
 * bookkeeping, no step of the method. */
MOC_API int moc_server_arena_overhead(int max_slots, size_t *bytes);

/* Queue a request: one fixed-source problem (geometry, tracks and cross
 * sections of the plan, source Q of Eq. 1) to be solved by the source
 * iteration of section 2.1 (FP32 sweep, stable exponential; opts->sweep_fp64
 * and opts->exp_mode must be 0).  The plan and q [n_fsr][G] are copied.
 * ENOMEM if the request could never fit the arena; EINVAL for bad input. */
MOC_API int moc_server_submit(moc_server *srv, const moc_plan *plan, const double *q,
                              const moc_solve_opts *opts, unsigned long long *ticket);

/* One step (one source iteration of section 2.1, Eqs. 3-4, for every active
 * request): admit waiting requests in arrival order while a slot is free
 * and the workspace fits (a request may be overtaken by smaller ones at most
 * 8 times), run one source iteration of every active request in one batched
 * launch sequence, and retire requests whose residual < tol (after the first
 * iteration) or that reached max_iters, as moc_solve stops.  While the batch
 * does not change, the next step is launched before this one's residuals are
 * read (the device applies the stopping rule itself and skips stopped
 * requests), so the call may return with one step still running on the
 * stream; that step's results are accounted by the next call.
 * *n_active / *n_queued (optional) report the state afterwards. */
MOC_API int moc_server_step(moc_server *srv, int *n_active, int *n_queued);

/* MOC_EBUSY while the request is queued or running.  Once it has retired:
 * copies its stats and (if flux_out) its Eq. 4 scalar flux [n_fsr][G]
 * (n must then be n_fsr * G, else EINVAL), releases it and
 * returns MOC_OK (converged) or MOC_ENOTCONV (stopped at max_iters). */
MOC_API int moc_server_poll(moc_server *srv, unsigned long long ticket, moc_stats *stats,
                            double *flux_out, size_t n);

/* Admission policy (serving bookkeeping, no step of the method): with
 * max_units > 0, queued requests are admitted in
 * arrival order only while the active requests hold at most max_units work
 * units (two per 2D track of each request; a request above the limit runs
 * alone).  Large requests then run close to first-come-first-served and small
 * ones share the GPU.  Default: 64 units per compute unit of the device;
 * 0: admit whatever fits the arena. */
MOC_API int moc_server_set_fill(moc_server *srv, long long max_units);

/* Non-releasing status check (serving bookkeeping): *done = 1 once the
 * request has retired (its result waits for moc_server_poll), 0 while queued
 * or running; EINVAL for an unknown ticket. */
MOC_API int moc_server_query(const moc_server *srv, unsigned long long ticket, int *done);

/* Text of the calling thread's last error ("" after success); valid until
 * that thread's next call.  Error reporting only. */
MOC_API const char *moc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MOC_H */
