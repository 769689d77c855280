/*
 * FP64 CPU oracle for fixed-source 3D method-of-characteristics transport.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that
 * the HIP path is checked against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it; the product path never does.
 * It shares no code, header, table or helper with the HIP library.
 *
 * What it computes (paper section 2): the discrete MOC operator with flat
 * sources (Eq. 3 segment attenuation, Eq. 4 track-length flux estimator) on
 * 3D characteristic tracks obtained by plain brute-force 3D ray tracing of
 * every track against every surface it crosses (cell planes, inclusion
 * circles, sector half-lines, axial planes), with explicit segment storage,
 * reflective links found by coordinate matching, and Jacobi source iteration.
 * The 3D track laydown (which lines exist) follows the z-stack construction
 * of Eq. 5 with the readings documented alongside the tests.
 */
#ifndef MOC_ORACLE_H
#define MOC_ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int nx, ny;
    double pitch, radius;
    int n_sectors;
    double height;
    int n_layers;
    int bc[6];                    /* x-, x+, y-, y+, z-, z+ : 0 vacuum, 1 reflective */
    const int *cell_material;     /* [ny*nx][2] = {inside, outside} */
    int n_azim, n_polar;
    double radial_spacing, axial_spacing;
    int n_groups, n_materials;
    const double *sigma_t;        /* [M][G] */
    const double *sigma_s;        /* [M][G][G], [m][g_from][g_to] */
} orc_problem;

typedef struct {
    long long n_fsr, n_regions, n_2d_tracks, n_3d_tracks, n_segments; /* segments: stored (undirected) */
    long long n_cycles;           /* directed 2D cycles */
    double dz;                    /* effective axial spacing */
    int traced;                   /* 1 when every 3D track was traced */
} orc_info;

typedef struct {
    int iters;
    double residual;
    double leakage;               /* sum over vacuum exits of W psi (last sweep) */
    double balance_lhs;           /* sum_j,g acc (last sweep)                     */
    double balance_rhs;           /* sum W psi_in(k-1) - sum W psi_out(k)         */
    double absorption, source;    /* physical totals at the last iterate          */
} orc_result;

typedef struct orc_model orc_model;

/* Gauss-Legendre nodes (ascending) and weights on [-1, 1]. */
int orc_gauss_legendre(int n, double *mu, double *w);

/* Build laydown, stacks and (when trace != 0) all 3D segments and links.
 * Returns 0 on success, <0 on invalid input. */
int orc_build(const orc_problem *p, int trace, int n_threads, orc_model **out);
void orc_free(orc_model *m);
void orc_get_info(const orc_model *m, orc_info *out);

/* Quadrature / laydown introspection (for pins). Arrays sized by the caller:
 * azim arrays [n_azim/2], polar arrays [n_polar], weight [n_azim/2][n_polar]. */
void orc_get_quadrature(const orc_model *m, double *phi_eff, double *dphi, double *spacing_eff,
                        int *nx_a, int *ny_a, double *mu, double *wpol, double *cot_eff,
                        double *weight);
/* 2D tracks: start/end points [n][4], length [n], azimuth [n], faces [n][2],
 * 2D links [n][2] as directed ids (2*t+d) of the successor of (t,fwd),(t,bwd),
 * chain coordinate a_t and direction sign sigma_t [n]. */
void orc_get_tracks2d(const orc_model *m, double *xy, double *len, int *azim, int *faces,
                      long long *link2d, double *chain, int *sigma);
/* z-stacks: for each (t, n) in Eq. 13 order: zeta, lowest line index, count. */
void orc_get_stacks(const orc_model *m, double *zeta, long long *i_lo, long long *count);

/* Segments of one stored 3D track (forward order).  Returns the segment count
 * (<= cap entries written) or <0 on error. */
long long orc_trace_track(const orc_model *m, long long track, int *fsr, double *len, long long cap);
/* 3D endpoints [6] and the forward/backward successors (directed ids, -1 vacuum).
 * Only valid after a traced build. */
int orc_track_info(const orc_model *m, long long track, double *p01, long long *succ);

/* Path length of a sample of stored 3D tracks, one direction each: adds
 * W l of every segment to wl [n_fsr] (FSR volumes restricted to the sample
 * are wl / (4 pi) per direction).  Works on untraced builds (tracks traced by
 * brute force).  <0 on error. */
int orc_sample_path_length(const orc_model *m, long long n_items, const long long *track,
                           double *wl, long long *n_seg_out);

/* 1 when directed track (track, dir) enters the box through a vacuum face
 * (its incoming angular flux is zero), 0 when every face it enters through
 * is reflective, <0 on error.  Works on untraced builds. */
int orc_entry_vacuum(const orc_model *m, long long track, int dir);

/* Number of segments of every stored 3D track [n_3d_tracks] (traced build). */
int orc_segment_counts(const orc_model *m, long long *counts);

/* Track-estimated FSR volumes [n_fsr] (valid after a traced build). */
int orc_volumes(const orc_model *m, double *vol);

/* Jacobi source iteration from phi = 0, psi = 0.  q is [n_fsr][G].
 * Stops when residual < tol or after max_iters.  phi_out [n_fsr][G].
 * res_hist (optional) receives the residual of every iteration. */
int orc_solve(const orc_model *m, const double *q, double tol, int max_iters,
              double *phi_out, double *res_hist, orc_result *res);

/* orc_solve with a choice of boundary-flux coupling.  chain 0: the flux
 * leaving a track enters its successor in the next sweep (Jacobi lag), and
 * inner >= 1 sweeps run per source iteration with the same source, the last
 * one's tallies giving the flux.  chain 1 (inner must be 1): each sweep
 * follows every chain of reflected tracks from its head, a track whose
 * start no other track continues into, with zero incoming flux, passing the
 * flux to the successor within the sweep (characteristic lines swept whole,
 * section 2.1, across reflective faces).  Returns -3 if some track lies on
 * a closed loop of reflections (no vacuum face on its chain). */
int orc_solve_ex(const orc_model *m, const double *q, double tol, int max_iters, int chain,
                 int inner, double *phi_out, double *res_hist, orc_result *res);

/* Number of chains of directed tracks and the longest chain (in tracks);
 * -3 if a closed loop of reflections exists (traced build). */
int orc_chain_info(const orc_model *m, long long *n_heads, long long *max_len);

/* Eigenvalue mode: power iteration on k-eff with fission source chi_g F_j / k,
 * F_j = sum_g nu_sigma_f phi_j,g (nu_sigma_f, chi [M][G]).  From phi = 1,
 * psi = 0, k = 1; the residual is the larger of the relative change of k and
 * the largest change of the normalised fission source over fissile FSRs;
 * stops when it is < tol (after the first iteration) or after max_iters.
 * phi_out [n_fsr][G] unnormalised, *k_out. */
int orc_solve_eigen(const orc_model *m, const double *nu_sigma_f, const double *chi, double tol,
                    int max_iters, double *phi_out, double *k_out, double *res_hist,
                    orc_result *res);

/* One sweep of a sample of directed 3D tracks, with given reduced source qhat
 * [n_fsr][G] and incoming angular flux psi_in [n_items][G].  Tallies
 * acc [n_fsr][G] += W * delta_psi of the sampled tracks only and returns each
 * track's outgoing flux psi_out [n_items][G].  Works on untraced builds: each
 * sampled track is traced on the fly by brute force. */
int orc_sweep_sample(const orc_model *m, long long n_items, const long long *track,
                     const int *dir, const double *qhat, const double *psi_in,
                     double *acc, double *psi_out, long long *n_seg_out);

/* Weight W = omega * A of 3D tracks on stored azimuth a, polar n. */
double orc_track_weight(const orc_model *m, long long track);

#ifdef __cplusplus
}
#endif
#endif
