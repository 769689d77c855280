// Device-side solver state: a plan bound to a caller workspace and stream.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "args.hpp"
#include "plan.hpp"

namespace moc {

struct SweepArgs;
struct FsrArgs;
struct SlotCtl;

// One batched source iteration of several problems (serving): device tables
// of per-problem descriptors and the work list of all their units.
struct BatchStep {
    const WinArgs *win_table;   // [n_slots]
    const FsrArgs *fsr_table;   // [n_slots]
    const int *blk_pre;         // [n_slots+1] 256-thread blocks per problem (prefix)
    const int *u_slot, *u_code; // [n_units]
    double *res_dev;            // [n_slots] residual of each problem
    SlotCtl *ctl;               // [n_slots] stopping rule and state of each problem (advanced by the step)
    int n_slots, n_units, fsr_blocks;
    int n_units_c1;             // units [0, n_units_c1) belong to problems with G <= 8
    int n_units_small;          // units [0, n_units_small) run in 256-thread workgroups
    size_t lds;                 // dynamic LDS of the 512-thread batched sweeps (max over problems)
    size_t lds_small;           // dynamic LDS of the 256-thread batched sweep
};
int launch_batch_step(const BatchStep &b, hipStream_t st);
// test hook: the sweep's F(tau) on the device for host values
int eval_attenuation(const float *tau, long long n, int exp_mode, float *out);
// the same without device allocation: staged through a fixed per-device array
// of kNoAllocMaxTau inputs and outputs
constexpr long long kNoAllocMaxTau = 1LL << 20;
int eval_attenuation_noalloc(const float *tau, long long n, int exp_mode, float *out);
// 2D segments per LDS window of the windowed sweep (0: does not fit)
int window_fit(const Plan &p, bool fp64);

void set_error(const std::string &e);
const char *last_error();
int fill_zero(void *p, size_t bytes, hipStream_t st);

double bundles_per_wave(const Plan &p, int Sw, int nt);

struct Solver {
    Layout lay;
    moc_plan_info info{};
    char *ws = nullptr;
    hipStream_t stream = nullptr;
    int P = 2, K = 1;
    double H = 1, h = 1;
    int bc[6] = {0, 0, 0, 0, 0, 0};
    int iter = 0;
    bool has_source = false;
    std::vector<float> sweep_ms;
    std::vector<hipEvent_t> events;
    int sw32 = 0, sw64 = 0;          // windowed sweep: 2D segments per window (0: direct path)
    int lstride = 1;                 // windowed sweep: line stride inside a bundle
    int walk = 0;                    // transport walk in use: 0 lockstep, 1 per-lane
    int walk_auto = 0;               // the plan's choice (set at upload)
    int sw256 = 0, sw1024 = 0;       // per-lane walk: windows of 256 / 1024-thread workgroups
    // per-lane walk: estimated 64-line bundles per wave in a window of the
    // 256 / 512 / 1024-thread workgroups (weighted by the window's lines)
    double bpw256 = 0, bpw512 = 0, bpw1024 = 0;
    int window_nt = 0;               // workgroup size the caller chose (0: automatic)
    int lane_nt = 512, lane_win = 0; // the single solver's per-lane sweep: workgroup size, window
    void choose_lane_window();
    int set_window(int threads);
    int lane_sw = 0;                 // per-lane walk: 2D segments per window of a 256-thread
                                     // workgroup (0: such windows are too short, 512 threads)
    void set_walk(int mode) { walk = mode == 0 ? walk_auto : mode - 1; }
    std::vector<long long> chunk_off, trk_off;
    std::vector<int> work_host;      // windowed-sweep work list (longest first)
    std::vector<float> work_cost;    // estimated cost of each work-list unit
    std::vector<double> track_work;  // estimated work per 2D track (lines x 2D segments)
    std::vector<int> cnt;

    // bind to a workspace: layout, upload, volumes, reset (returns moc_status)
    int init(const Plan &p, char *workspace, size_t ws_bytes, hipStream_t st);
    SweepArgs sweep_args(int fp64, int exp_mode) const;
    FsrArgs fsr_args() const;
    int upload(const Plan &p);
    int compute_volumes();
    void launch_sweep(SweepArgs a, bool fp64, const int *units = nullptr, int n_units = 0,
                      const int *filt_n = nullptr, const long long *filt_i0 = nullptr);
    bool lane_path(const SweepArgs &a, bool fp64) const;   // the per-lane FP32 transport sweep
    WinArgs lane_args(const SweepArgs &a) const;
    int resident_workgroups() const;
    // schedule of the work units (paper section 4.3): order 0 longest first,
    // 1 natural (2D track order), 2 by decreasing work in groups of the
    // resident workgroup count, every other group reversed; persistent: a
    // grid of resident workgroups, each sweeping units b, b + grid, ...
    int order = 0;
    int persistent = 0;
    int set_schedule(int order, int persistent);
    // bundles of a window: -1 automatic (dynamic in 1024-thread windows),
    // 0 static (wave w takes w, w + waves, ...), 1 dynamic (an LDS counter)
    int bundles = -1;
    bool dyn_bundles() const;
    // chain-line sweep: the flux leaving a line through a reflective side
    // face enters its continuation within the same sweep (vacuum top and
    // bottom faces; the per-lane FP32 sweep only).  0 off, 1 on
    int chain = 0;
    int64_t n_chseg = 0;
    int chain_cap = 0;               // lines per stack of a carry buffer
    bool chain_only = false;         // workspace without boundary buffers
    int set_chain(int on);
    int upload_work_list();
    // stored-segment (EXP) sweep (paper section 4.2): the recorded pieces of
    // the units with the most pieces, replayed; the other units on the fly
    int exp_units = 0, otf_units = 0;
    int *d_exp_work = nullptr, *d_otf_work = nullptr;
    unsigned *d_exp_tbase = nullptr, *d_exp_table = nullptr;
    Piece *d_exp_data = nullptr;
    int store_segments(char *buf, size_t bytes, moc_store_info *out);
    void drop_store() {
        exp_units = otf_units = 0;
        d_exp_work = d_otf_work = nullptr;
        d_exp_tbase = d_exp_table = nullptr;
        d_exp_data = nullptr;
    }
    int window_size(bool fp64) const { return fp64 ? sw64 : sw32; }
    WinArgs win_args_batched() const;   // descriptor of the batched sweep (even orientation)
    size_t win_lds() const;
    size_t lane_lds() const;            // LDS of a 256-thread per-lane window (lane_sw)
    int reset();
    int iterate(int nit, const moc_solve_opts &o, bool time_sweep);
    // One source iteration for moc_solve: on a non-default stream a captured
    // graph per boundary-buffer parity (source update, sweep between two
    // timing events, finalize, residual fold, 8-byte copy to pinned host
    // memory); else the same launches one by one.  *res receives the residual.
    int solve_step(const moc_solve_opts &o, double *res);
    hipGraphExec_t step_exec[2] = {nullptr, nullptr};
    int step_key = -1;               // sweep precision / exp mode / walk the graphs were built for
    bool step_graphs_failed = false; // capture unsupported: launch one by one
    double *h_res = nullptr;         // pinned: the folded residual of the last step
    hipEvent_t step_ev[2] = {nullptr, nullptr};
    void drop_step_graphs();
    int read_stats(moc_stats *st);
    int read_residual(double *r);
    int n_materials = 0;
    // eigenvalue mode (power iteration on k-eff); nusf, chi host [M][G]
    int solve_eigen(const double *nusf, const double *chi, const moc_solve_opts &o, double *k_out,
                    double *res_out, int *iters_out);
    int sweep_items(long long n_items, const long long *items, const double *qhat,
                    const double *psi_in, int fp64, double *acc_out, double *psi_out);
    int trace_tracks(long long n, const long long *ids, int cap, int *fsr, double *len,
                     int *count);
    // incoming boundary flux of the next sweep for directed slots (host out [n][G])
    int gather_boundary(long long n, const long long *slots, double *out);
    ~Solver();
};

}  // namespace moc

struct moc_solver {
    moc::Solver s;
};
