// C ABI entry points (declared in include/moc.h): argument checking, plan and
// solver lifetime, and the source-iteration driver.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "plan.hpp"
#include "solver.hpp"

using moc::set_error;

namespace {

int fail(int code, const std::string &msg) {
    set_error(msg);
    return code;
}

}  // namespace

extern "C" {

const char *moc_last_error(void) { return moc::last_error(); }

int moc_plan_create(const moc_geometry *geom, const moc_tracking *trk, const moc_xs *xs,
                    moc_plan **out) {
    if (!out) return fail(MOC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!geom || !trk || !xs) return fail(MOC_EINVAL, "NULL argument");
    moc_plan *p = new (std::nothrow) moc_plan();
    if (!p) return fail(MOC_ENOMEM, "host allocation failed");
    std::string err;
    try {
        err = p->p.build(*geom, *trk, *xs);
    } catch (const std::bad_alloc &) {
        delete p;
        return fail(MOC_ENOMEM, "host allocation failed while planning");
    }
    if (!err.empty()) {
        delete p;
        return fail(MOC_EINVAL, err);
    }
    *out = p;
    set_error("");
    return MOC_OK;
}

int moc_plan_query(const moc_plan *plan, moc_plan_info *out) {
    if (!plan || !out) return fail(MOC_EINVAL, "NULL argument");
    *out = plan->p.info();
    return MOC_OK;
}

void moc_plan_destroy(moc_plan *plan) { delete plan; }

int moc_plan_quadrature(const moc_plan *plan, double *phi, double *dphi, double *spacing,
                        double *cot, double *weight) {
    if (!plan) return fail(MOC_EINVAL, "NULL plan");
    const moc::Plan &p = plan->p;
    for (int a = 0; a < p.A2; ++a) {
        if (phi) phi[a] = p.phi[a];
        if (dphi) dphi[a] = p.dphi[a];
        if (spacing) spacing[a] = p.deff[a];
    }
    for (size_t i = 0; i < p.cot.size(); ++i) {
        if (cot) cot[i] = p.cot[i];
        if (weight) weight[i] = p.wgt[i];
    }
    return MOC_OK;
}

int moc_plan_tracks2d(const moc_plan *plan, double *xy, double *length, int *azim,
                      long long *link, double *chain, int *sigma) {
    if (!plan) return fail(MOC_EINVAL, "NULL plan");
    const moc::Plan &p = plan->p;
    for (int64_t t = 0; t < p.n2d; ++t) {
        if (xy) {
            xy[4 * t] = p.x0[t];
            xy[4 * t + 1] = p.y0[t];
            xy[4 * t + 2] = p.x1[t];
            xy[4 * t + 3] = p.y1[t];
        }
        if (length) length[t] = p.L[t];
        if (azim) azim[t] = p.az[t];
        if (link) {
            link[2 * t] = p.link[2 * t];
            link[2 * t + 1] = p.link[2 * t + 1];
        }
        if (chain) chain[t] = p.chain[t];
        if (sigma) sigma[t] = p.sig[t];
    }
    return MOC_OK;
}

int moc_plan_stacks(const moc_plan *plan, double *zeta, long long *i_lo, long long *count) {
    if (!plan) return fail(MOC_EINVAL, "NULL plan");
    const moc::Plan &p = plan->p;
    for (int64_t s = 0; s < p.n_stacks; ++s) {
        if (zeta) zeta[s] = p.zeta[s];
        if (i_lo) i_lo[s] = p.ilo[s];
        if (count) count[s] = p.cnt[s];
    }
    return MOC_OK;
}

int moc_plan_chain(const moc_plan *plan, long long *first, int *k, int *nk, double *lc, int *code,
                   double *u) {
    if (!plan) return fail(MOC_EINVAL, "NULL plan");
    const moc::Plan &p = plan->p;
    for (int64_t s = 0; s < p.n_chseg; ++s) {
        if (k) k[s] = p.ch_k[s];
        if (nk) nk[s] = p.ch_nk[s];
        if (lc) lc[s] = p.ch_lc[s];
    }
    for (int64_t s = 0; s <= p.n_chseg; ++s)
        if (first) first[s] = p.ch_first[s];
    for (size_t i = 0; i < p.ch_code.size(); ++i) {
        if (code) code[i] = p.ch_code[i];
        if (u) u[i] = p.ch_u[i];
    }
    return MOC_OK;
}

int moc_plan_segments2d(const moc_plan *plan, double *pos, int *region, long long *first) {
    if (!plan) return fail(MOC_EINVAL, "NULL plan");
    const moc::Plan &p = plan->p;
    for (size_t k = 0; k < p.seg_pos.size(); ++k) {
        if (pos) pos[k] = p.seg_pos[k];
        if (region) region[k] = p.seg_reg[k];
    }
    if (first)
        for (int64_t t = 0; t <= p.n2d; ++t) first[t] = p.seg_first[t];
    return MOC_OK;
}

int moc_plan_chunk(const moc_plan *plan, long long chunk, long long *first_track, int *n_tracks) {
    if (!plan) return fail(MOC_EINVAL, "NULL plan");
    const moc::Plan &p = plan->p;
    if (chunk < 0 || chunk >= p.n_chunks) return fail(MOC_EINVAL, "chunk out of range");
    int64_t lo = 0, hi = p.n_stacks;
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) / 2;
        if (p.chunk_off[mid] <= chunk) lo = mid;
        else hi = mid;
    }
    int64_t z0 = (chunk - p.chunk_off[lo]) * p.T;
    int64_t n = std::min<int64_t>(p.T, p.cnt[lo] - z0);
    if (first_track) *first_track = p.trk_off[lo] + z0;
    if (n_tracks) *n_tracks = (int)n;
    return MOC_OK;
}

int moc_solver_create(const moc_plan *plan, void *dev_workspace, size_t ws_bytes, void *stream,
                      moc_solver **out) {
    if (!out) return fail(MOC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!plan || !dev_workspace) return fail(MOC_EINVAL, "NULL plan or workspace");
    const moc::Plan &p = plan->p;
    moc_solver *sv = new (std::nothrow) moc_solver();
    if (!sv) return fail(MOC_ENOMEM, "host allocation failed");
    int rc = sv->s.init(p, static_cast<char *>(dev_workspace), ws_bytes, static_cast<hipStream_t>(stream));
    if (rc) {
        delete sv;
        return rc;
    }
    *out = sv;
    return MOC_OK;
}

void moc_solver_destroy(moc_solver *s) { delete s; }

int moc_set_source(moc_solver *sv, const double *q, size_t n) {
    if (!sv || !q) return fail(MOC_EINVAL, "NULL argument");
    moc::Solver &s = sv->s;
    const size_t need = (size_t)s.info.n_fsr * s.info.n_groups;
    if (n != need) return fail(MOC_EINVAL, "source size must be n_fsr * n_groups");
    for (size_t i = 0; i < n; ++i)
        if (!(q[i] >= 0) || !std::isfinite(q[i])) return fail(MOC_EINVAL, "source must be finite and >= 0");
    hipError_t e = hipMemcpyAsync(s.ws + s.lay.off_q, q, n * 8, hipMemcpyHostToDevice, s.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
    if (e != hipSuccess) return fail(MOC_EDEVICE, hipGetErrorString(e));
    s.has_source = true;
    return MOC_OK;
}

static int check_opts(const moc_solve_opts *o) {
    if (!o) return fail(MOC_EINVAL, "NULL options");
    if (o->max_iters < 1) return fail(MOC_EINVAL, "max_iters must be >= 1");
    if (!(o->tol >= 0)) return fail(MOC_EINVAL, "tol must be >= 0");
    if (o->exp_mode != 0 && o->exp_mode != 1) return fail(MOC_EINVAL, "exp_mode must be 0 or 1");
    return MOC_OK;
}

int moc_reset(moc_solver *sv) {
    if (!sv) return fail(MOC_EINVAL, "NULL solver");
    return sv->s.reset();
}

int moc_solver_set_walk(moc_solver *sv, int walk) {
    if (!sv) return fail(MOC_EINVAL, "NULL solver");
    if (walk < 0 || walk > 2) return fail(MOC_EINVAL, "walk must be 0 (automatic), 1 (lockstep) or 2 (per-lane)");
    sv->s.set_walk(walk);
    return MOC_OK;
}

int moc_solver_store_segments(moc_solver *sv, void *dev_store, size_t store_bytes, moc_store_info *info) {
    if (!sv) return fail(MOC_EINVAL, "NULL solver");
    if (dev_store && (reinterpret_cast<uintptr_t>(dev_store) & 255) != 0)
        return fail(MOC_EINVAL, "store must be 256-byte aligned");
    return sv->s.store_segments(static_cast<char *>(dev_store), dev_store ? store_bytes : 0, info);
}

int moc_solver_set_schedule(moc_solver *sv, int order, int persistent) {
    if (!sv) return fail(MOC_EINVAL, "NULL solver");
    if (order < 0 || order > 2) return fail(MOC_EINVAL, "order must be 0, 1 or 2");
    if (persistent != 0 && persistent != 1) return fail(MOC_EINVAL, "persistent must be 0 or 1");
    return sv->s.set_schedule(order, persistent);
}

int moc_solver_set_bundles(moc_solver *sv, int mode) {
    if (!sv) return fail(MOC_EINVAL, "NULL solver");
    if (mode < -1 || mode > 1) return fail(MOC_EINVAL, "mode must be -1 (automatic), 0 or 1");
    sv->s.bundles = mode;
    sv->s.drop_step_graphs();
    return MOC_OK;
}

int moc_solver_set_chain(moc_solver *sv, int on) {
    if (!sv) return fail(MOC_EINVAL, "NULL solver");
    if (on != 0 && on != 1) return fail(MOC_EINVAL, "on must be 0 or 1");
    if (sv->s.chain_only && on == 0) return fail(MOC_EINVAL, "a chain-only solver cannot leave chain mode");
    if (sv->s.set_chain(on))
        return fail(MOC_EINVAL, "the chain-line sweep needs vacuum top and bottom faces, an even polar "
                                "count and the per-lane FP32 sweep (at most 8 groups)");
    return MOC_OK;
}

int moc_solver_set_window(moc_solver *sv, int threads) {
    if (!sv) return fail(MOC_EINVAL, "NULL solver");
    if (threads != 0 && threads != 256 && threads != 512 && threads != 1024)
        return fail(MOC_EINVAL, "threads must be 0 (automatic), 256, 512 or 1024");
    if (sv->s.set_window(threads)) return fail(MOC_EINVAL, "no window of that workgroup size fits the LDS");
    return MOC_OK;
}

int moc_solver_window(const moc_solver *sv, int *threads, int *segments) {
    if (!sv) return fail(MOC_EINVAL, "NULL solver");
    if (threads) *threads = sv->s.lane_nt;
    if (segments) *segments = sv->s.lane_win;
    return MOC_OK;
}

int moc_solver_walk(const moc_solver *sv, int *walk) {
    if (!sv || !walk) return fail(MOC_EINVAL, "NULL argument");
    *walk = sv->s.walk + 1;
    return MOC_OK;
}

int moc_iterate(moc_solver *sv, int n, const moc_solve_opts *opts, moc_stats *stats) {
    if (!sv) return fail(MOC_EINVAL, "NULL solver");
    if (n < 1) return fail(MOC_EINVAL, "n must be >= 1");
    moc_solve_opts o{0.0, 1, 0, 0};
    if (opts) {
        int rc = check_opts(opts);
        if (rc) return rc;
        o = *opts;
    }
    int rc = sv->s.iterate(n, o, stats != nullptr);
    if (rc) return rc;
    if (stats) return sv->s.read_stats(stats);
    return MOC_OK;
}

int moc_solve(moc_solver *sv, const moc_solve_opts *opts, moc_stats *stats) {
    if (!sv) return fail(MOC_EINVAL, "NULL solver");
    int rc = check_opts(opts);
    if (rc) return rc;
    moc::Solver &s = sv->s;
    rc = s.reset();
    if (rc) return rc;
    double res = 1.0;
    for (int k = 0; k < opts->max_iters; ++k) {
        rc = s.solve_step(*opts, &res);
        if (rc) return rc;
        if (res < opts->tol) break;
    }
    if (stats) {
        rc = s.read_stats(stats);
        if (rc) return rc;
    }
    return res < opts->tol ? MOC_OK : MOC_ENOTCONV;
}

int moc_solve_eigen(moc_solver *sv, const double *nu_sigma_f, const double *chi,
                    const moc_solve_opts *opts, double *k_eff, moc_stats *stats) {
    if (!sv || !nu_sigma_f || !chi || !k_eff) return fail(MOC_EINVAL, "NULL argument");
    int rc = check_opts(opts);
    if (rc) return rc;
    moc::Solver &s = sv->s;
    const size_t mg = (size_t)s.n_materials * s.info.n_groups;
    bool any = false;
    for (size_t i = 0; i < mg; ++i) {
        if (!(nu_sigma_f[i] >= 0) || !std::isfinite(nu_sigma_f[i]) || !(chi[i] >= 0) || !std::isfinite(chi[i]))
            return fail(MOC_EINVAL, "nu_sigma_f and chi must be finite and >= 0");
        any = any || nu_sigma_f[i] > 0;
    }
    if (!any) return fail(MOC_EINVAL, "nu_sigma_f is zero everywhere");
    double k = 0.0, res = 1.0;
    int iters = 0;
    rc = s.solve_eigen(nu_sigma_f, chi, *opts, &k, &res, &iters);
    if (rc) return rc;
    *k_eff = k;
    if (stats) {
        rc = s.read_stats(stats);
        if (rc) return rc;
        stats->iters = iters;
        stats->residual = res;
    }
    return (iters > 1 && res < opts->tol) ? MOC_OK : MOC_ENOTCONV;
}

int moc_get_flux(const moc_solver *sv, double *host_out, size_t n) {
    if (!sv || !host_out) return fail(MOC_EINVAL, "NULL argument");
    const moc::Solver &s = sv->s;
    if (n != (size_t)s.info.n_fsr * s.info.n_groups) return fail(MOC_EINVAL, "size must be n_fsr * n_groups");
    hipError_t e = hipMemcpyAsync(host_out, s.ws + s.lay.off_phi, n * 8, hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
    if (e != hipSuccess) return fail(MOC_EDEVICE, hipGetErrorString(e));
    return MOC_OK;
}

int moc_get_volumes(const moc_solver *sv, double *host_out, size_t n) {
    if (!sv || !host_out) return fail(MOC_EINVAL, "NULL argument");
    const moc::Solver &s = sv->s;
    if (n != (size_t)s.info.n_fsr) return fail(MOC_EINVAL, "size must be n_fsr");
    hipError_t e = hipMemcpyAsync(host_out, s.ws + s.lay.off_vol, n * 8, hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
    if (e != hipSuccess) return fail(MOC_EDEVICE, hipGetErrorString(e));
    return MOC_OK;
}

int moc_flux_device_ptr(const moc_solver *sv, const double **dev) {
    if (!sv || !dev) return fail(MOC_EINVAL, "NULL argument");
    *dev = reinterpret_cast<const double *>(sv->s.ws + sv->s.lay.off_phi);
    return MOC_OK;
}

int moc_sweep_items(moc_solver *sv, long long n_items, const long long *items, const double *qhat,
                    const double *psi_in, int sweep_fp64, double *acc_out, double *psi_out) {
    if (!sv || !items || !qhat || !psi_in || !acc_out || !psi_out) return fail(MOC_EINVAL, "NULL argument");
    moc::Solver &s = sv->s;
    for (long long i = 0; i < n_items; ++i)
        if (items[i] < 0 || items[i] >= 2 * s.info.n_chunks) return fail(MOC_EINVAL, "work item out of range");
    return s.sweep_items(n_items, items, qhat, psi_in, sweep_fp64, acc_out, psi_out);
}

int moc_get_reduced_source(const moc_solver *sv, int fp64, double *host_out, size_t n) {
    if (!sv || !host_out) return fail(MOC_EINVAL, "NULL argument");
    if (fp64 != 0 && fp64 != 1) return fail(MOC_EINVAL, "fp64 must be 0 or 1");
    const moc::Solver &s = sv->s;
    if (n != (size_t)s.info.n_fsr * s.info.n_groups) return fail(MOC_EINVAL, "size must be n_fsr * n_groups");
    hipError_t e;
    if (fp64) {
        e = hipMemcpyAsync(host_out, s.ws + s.lay.off_qhat64, n * 8, hipMemcpyDeviceToHost, s.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
    } else {
        std::vector<float> q32;
        try {
            q32.resize(n);
        } catch (const std::bad_alloc &) {
            return fail(MOC_ENOMEM, "host allocation failed");
        }
        e = hipMemcpyAsync(q32.data(), s.ws + s.lay.off_qhat32, n * 4, hipMemcpyDeviceToHost, s.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
        if (e == hipSuccess)
            for (size_t i = 0; i < n; ++i) host_out[i] = q32[i];
    }
    if (e != hipSuccess) return fail(MOC_EDEVICE, hipGetErrorString(e));
    return MOC_OK;
}

int moc_get_boundary_flux(const moc_solver *sv, long long n, const long long *slots, double *out) {
    if (!sv || (n > 0 && (!slots || !out))) return fail(MOC_EINVAL, "NULL argument");
    if (n < 0) return fail(MOC_EINVAL, "n must be >= 0");
    const moc::Solver &s = sv->s;
    for (long long i = 0; i < n; ++i)
        if (slots[i] < 0 || slots[i] >= 2 * s.info.n_3d_tracks) return fail(MOC_EINVAL, "slot out of range");
    return const_cast<moc::Solver &>(s).gather_boundary(n, slots, out);
}

int moc_trace_tracks(moc_solver *sv, long long n, const long long *track_ids, int cap, int *fsr_out,
                     double *len_out, int *count_out) {
    if (!sv || !track_ids || !fsr_out || !len_out || !count_out) return fail(MOC_EINVAL, "NULL argument");
    if (cap < 1 || cap > 65536) return fail(MOC_EINVAL, "cap must be in [1, 65536]");
    moc::Solver &s = sv->s;
    if ((size_t)cap * 12 + 16 + 1024 > s.lay.scratch_bytes) return fail(MOC_EINVAL, "cap too large for the scratch area");
    for (long long i = 0; i < n; ++i)
        if (track_ids[i] < 0 || track_ids[i] >= s.info.n_3d_tracks) return fail(MOC_EINVAL, "track id out of range");
    return s.trace_tracks(n, track_ids, cap, fsr_out, len_out, count_out);
}

int moc_eval_attenuation(const float *tau, long long n, int exp_mode, float *out) {
    if (n < 0 || (n > 0 && (!tau || !out))) return fail(MOC_EINVAL, "NULL argument or n < 0");
    if (exp_mode != 0 && exp_mode != 1) return fail(MOC_EINVAL, "exp_mode must be 0 or 1");
    if (n > (1LL << 28)) return fail(MOC_EINVAL, "n too large (at most 2^28)");
    for (long long i = 0; i < n; ++i)
        if (!(tau[i] >= 0.0f) || !std::isfinite(tau[i])) return fail(MOC_EINVAL, "tau must be finite and >= 0");
    return moc::eval_attenuation(tau, n, exp_mode, out);
}

int moc_eval_attenuation_noalloc(const float *tau, long long n, int exp_mode, float *out) {
    if (n < 0 || (n > 0 && (!tau || !out))) return fail(MOC_EINVAL, "NULL argument or n < 0");
    if (exp_mode != 0 && exp_mode != 1) return fail(MOC_EINVAL, "exp_mode must be 0 or 1");
    if (n > moc::kNoAllocMaxTau)
        return fail(MOC_EINVAL, "n exceeds the fixed staging capacity (2^20 values per call)");
    for (long long i = 0; i < n; ++i)
        if (!(tau[i] >= 0.0f) || !std::isfinite(tau[i])) return fail(MOC_EINVAL, "tau must be finite and >= 0");
    return moc::eval_attenuation_noalloc(tau, n, exp_mode, out);
}

}  // extern "C"
