// Kernel argument records shared by the kernels and the host code that fills
// them (plain data: device pointers into one problem's workspace and sizes).
#pragma once

namespace moc {

struct SweepArgs {
    const double *cot, *icot, *secl, *wgt;       // [A2][P]: cot, 1/cot, 1/sin, weight
    const double *t_len;                          // [n2d]
    const int *t_first, *t_meta, *t_link;         // [n2d+1], [n2d], [2*n2d]
    const double *seg_pos;                        // [nseg]
    const int *seg_reg, *reg_mat;                 // [nseg], [n_regions]
    const double *zeta;                           // [n_stacks]
    const long long *ilo;                         // [n_stacks]
    const int *cnt;                               // [n_stacks]
    const long long *trk_off, *chunk_off;         // [n_stacks+1]
    const void *sigt;                             // [M][G] float or double
    const double *sigt64;                         // [M][G] double (always)
    const void *qhat;                             // [n_fsr][G] float or double
    double *acc;                                  // [n_fsr][G]
    void *psi_in;                                 // boundary buffer read this sweep
    void *psi_out;                                // boundary buffer written (may be null)
    const double *psi_entry;                      // per (item, lane) incoming flux (test hook)
    double *psi_exit;                             // per (item, lane) outgoing flux (test hook)
    const long long *items;                       // explicit work list or null
    long long n_items;
    long long n_stacks;
    double *scal;
    double H, h, inv_h, dz, inv_dz;
    int G, P, K, T;
    int C, GL;                                    // group chunks across lanes, groups per lane
    int bc[6];
    int exp_mode;
    int mode;                                     // 0 sweep, 1 volume tally
};

struct WinArgs {
    SweepArgs s;
    const int *work;          // work unit codes 2*t + dir (longest first)
    const int *filt_n;        // test hook: only this polar stack per unit (or null)
    const long long *filt_i0; // test hook: only lines [i0, i0+T) of it
    int Sw;                   // 2D segments per window
    int lstride;              // line stride inside a bundle (1: consecutive lines)
    int walk;                 // transport walk of the FP32 one-chunk sweep: 0 lockstep, 1 per-lane
    int small_wg;             // per-lane walk in 256-thread workgroups (Sw sized for them)
};

// Per-problem control of a batched step: the stopping rule and the state the
// step advances (completed iterations, done once stopped).
struct SlotCtl {
    double tol;
    int max_iters;
    int iters;
    int done;
    int pad_;
};

struct FsrArgs {
    const double *q, *sigt, *sigs, *vol;
    const int *reg_mat;
    double *phi, *acc, *qhat64;
    float *qhat32;
    double *scal;
    long long n;        // n_fsr * G
    int G, K;
};

}  // namespace moc
