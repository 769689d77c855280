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
    const float *seg_st;                          // [nseg][G] Sigma_t log2(e) of each 2D segment (FP32)
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

// One recorded piece of the stored-segment (EXP) sweep: the LDS tally /
// reduced-source row of the piece (bits 0-15) and its 2D segment in the window
// (bits 16-31), and its 3D length (FP32; 0 for a piece below the minimum
// length, -1 for a lane whose line has left the window).
struct Piece {
    unsigned idx;
    float len;
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
    int big_wg;               // per-lane walk in 1024-thread workgroups (Sw sized for them)
    int dyn_bundles;          // windowed sweep: waves take a window's bundles dynamically
    int persist_units;        // > 0: persistent grid, workgroup b sweeps units b, b + grid, ...
    // stored-segment (EXP) sweep of the per-lane walk
    int exp_pass;             // store pass: 1 count, 2 step table, 3 record
    unsigned long long *exp_count;   // count pass: [launch unit][2] = {wave steps, bundle windows}
    const unsigned *exp_tbase;       // first step-table entry of each unit of the launch
    unsigned *exp_table;             // per (unit, window, bundle): steps, then their exclusive prefix
    Piece *exp_data;                 // recorded pieces [wave step][64 lanes]
    // chain-line sweep: each workgroup takes segments (chain_ctr, a counter
    // from zero) and sweeps their items in order (see Plan::ch_*)
    int chain_nseg, chain_cap;
    const int *chain_first, *chain_code, *chain_k, *chain_nk;
    const double *chain_u, *chain_lc;
    unsigned *chain_ctr;
    void *chain_carry;                // per workgroup: [2 parities][P stacks][chain_cap][G] fluxes
};

// The lines of one chain-sweep item: segment k of nk of a traversal of
// length lc, the unit's unrolled start u, and the workgroup's carries.
struct ChainItem {
    int seg, nseg;
    int cap;        // lines per stack in a carry buffer
    void *cur;      // this item's carry buffer [P stacks][cap][G]
    void *next;     // the next item's
    double u, lc;
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
