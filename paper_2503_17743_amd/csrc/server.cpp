// Continuous batching of independent fixed-source solves on one GPU.
//
// Requests wait in arrival order.  A request is admitted when a slot is free
// and its workspace fits in the caller's device arena (first-fit; a request
// that does not fit may be overtaken by later, smaller ones a bounded number
// of times).  Every step runs one source iteration of every active request
// with one batched launch sequence (per-problem descriptor tables, one work
// list of all their (2D track, direction) units), captured in a HIP graph
// that is re-captured only when the set of active requests changes.  A
// request retires when its residual drops below its tolerance or it reaches
// max_iters; its flux stays on the device until it is polled.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "args.hpp"
#include "plan.hpp"
#include "solver.hpp"

namespace moc {
namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxBypass = 8;          // times a waiting request may be overtaken
constexpr size_t kUnitCap = 1 << 22;   // work units of all active requests together

size_t align_up(size_t n) { return (n + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over [0, size) of the caller's arena.
struct Arena {
    std::map<size_t, size_t> free_;   // offset -> size
    void init(size_t base, size_t size) {
        free_.clear();
        if (size) free_[base] = size;
    }
    bool alloc(size_t n, size_t &off) {
        n = align_up(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                off = it->first;
                const size_t rem = it->second - n, o2 = it->first + n;
                free_.erase(it);
                if (rem) free_[o2] = rem;
                return true;
            }
        }
        return false;
    }
    bool can_alloc(size_t n) const {
        n = align_up(n);
        for (const auto &f : free_)
            if (f.second >= n) return true;
        return false;
    }
    void release(size_t off, size_t n) {
        n = align_up(n);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

enum { QUEUED = 0, RUNNING = 1, DONE = 2 };

struct Request {
    unsigned long long ticket = 0;
    std::unique_ptr<Plan> plan;        // dropped once the request is admitted
    std::vector<double> q;
    moc_solve_opts opts{};
    int state = QUEUED;
    size_t off = 0, bytes = 0;
    Solver solver;
    long long units = 0;
    int iters = 0;
    double residual = 1.0;
    moc_stats stats{};
    bool converged = false;
    bool stopped = false;              // met the stopping rule (retired at the next drain)
    int bypassed = 0;
};

}  // namespace

struct Server {
    char *arena = nullptr;
    size_t arena_bytes = 0;
    size_t usable_bytes = 0;    // arena bytes after the server tables
    int max_slots = 1;
    long long fill_units = 0;   // admission stops at this many active work units (0: no limit)
    hipStream_t stream = nullptr;
    Arena alloc;
    unsigned long long next_ticket = 1;
    std::deque<Request *> queue;
    std::vector<Request *> active;
    std::map<unsigned long long, std::unique_ptr<Request>> all;
    // device tables (carved from the front of the arena)
    WinArgs *d_win = nullptr;
    FsrArgs *d_fsr = nullptr;
    int *d_blk = nullptr, *d_uslot = nullptr, *d_ucode = nullptr;
    SlotCtl *d_ctl = nullptr;
    double *d_res = nullptr;
    // pinned host staging; residuals in two halves, one per step in flight
    WinArgs *h_win = nullptr;
    FsrArgs *h_fsr = nullptr;
    SlotCtl *h_ctl = nullptr;
    double *h_res = nullptr;
    // current batch: two graphs of the same step, writing the two residual halves
    BatchStep batch{};
    bool dirty = true;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipEvent_t done_ev[2] = {nullptr, nullptr};
    // steps in flight: the oldest one's half (-1: none) and the next half to use
    int inflight = -1;
    int next_half = 0;

    ~Server() {
        for (int b = 0; b < 2; ++b) {
            if (exec[b]) (void)hipGraphExecDestroy(exec[b]);
            if (graph[b]) (void)hipGraphDestroy(graph[b]);
            if (done_ev[b]) (void)hipEventDestroy(done_ev[b]);
        }
        if (h_win) (void)hipHostFree(h_win);
        if (h_fsr) (void)hipHostFree(h_fsr);
        if (h_ctl) (void)hipHostFree(h_ctl);
        if (h_res) (void)hipHostFree(h_res);
    }

    int admit();
    bool admissible() const;
    int rebuild();
    int launch(int half);
    int collect(int half, bool *changed);
    int step(int *n_active, int *n_queued);
    void retire(Request *r);
};

#define SRV_HIPCHK(x)                                                        \
    do {                                                                     \
        hipError_t e_ = (x);                                                 \
        if (e_ != hipSuccess) {                                              \
            set_error(std::string(#x) + ": " + hipGetErrorString(e_));       \
            return MOC_EDEVICE;                                              \
        }                                                                    \
    } while (0)

int Server::admit() {
    long long units = 0;
    for (Request *r : active) units += r->units;
    bool blocked = false;
    for (auto it = queue.begin(); it != queue.end();) {
        Request *r = *it;
        if ((int)active.size() >= max_slots) break;
        // fill target: keep arrival order and stop once the batch holds enough
        // work to fill the GPU (a request larger than the target runs alone)
        if (fill_units > 0 && !active.empty() && units + r->units > fill_units) break;
        size_t off = 0;
        const bool fits = (units + r->units <= (long long)kUnitCap) && alloc.alloc(r->bytes, off);
        if (!fits) {
            // a request that keeps being overtaken stops everything behind it
            if (r->bypassed >= kMaxBypass) blocked = true;
            ++it;
            if (blocked) break;
            continue;
        }
        for (auto jt = queue.begin(); jt != it; ++jt) ++(*jt)->bypassed;
        int rc = r->solver.init(*r->plan, arena + off, r->bytes, stream);
        if (!rc) {
            hipError_t e = hipMemcpyAsync(r->solver.ws + r->solver.lay.off_q, r->q.data(),
                                          r->q.size() * 8, hipMemcpyHostToDevice, stream);
            if (e == hipSuccess) e = hipStreamSynchronize(stream);
            if (e != hipSuccess) {
                set_error(hipGetErrorString(e));
                rc = MOC_EDEVICE;
            }
        }
        if (rc) {
            alloc.release(off, r->bytes);
            return rc;
        }
        r->off = off;
        r->state = RUNNING;
        r->plan.reset();
        r->q.clear();
        r->q.shrink_to_fit();
        units += r->units;
        active.push_back(r);
        it = queue.erase(it);
        dirty = true;
    }
    return MOC_OK;
}

// Whether admit() would take a queued request now (the same checks, no
// allocation).
bool Server::admissible() const {
    if (queue.empty() || (int)active.size() >= max_slots) return false;
    long long units = 0;
    for (const Request *r : active) units += r->units;
    for (const Request *r : queue) {
        if (fill_units > 0 && !active.empty() && units + r->units > fill_units) return false;
        if (units + r->units <= (long long)kUnitCap && alloc.can_alloc(r->bytes)) return true;
        if (r->bypassed >= kMaxBypass) return false;
    }
    return false;
}

// Work list, block prefix, descriptor tables and graphs of the current set of
// active requests (called with no step in flight).
int Server::rebuild() {
    const int n = (int)active.size();
    std::vector<int> blk(n + 1, 0);
    // one-chunk problems with shallow stacks sweep in 256-thread workgroups
    // (their own launch, shorter windows), like their one-at-a-time solves
    auto small = [&](int i) {
        const Solver &s = active[i]->solver;
        return s.info.n_groups <= kGL && s.lane_sw >= 1;
    };
    size_t lds = 0, lds_small = 0;
    for (int i = 0; i < n; ++i) {
        Solver &s = active[i]->solver;
        const long long nfg = (long long)s.info.n_fsr * s.info.n_groups;
        blk[i + 1] = blk[i] + (int)((nfg + 255) / 256);
        if (small(i)) lds_small = std::max(lds_small, s.lane_lds());
        else lds = std::max(lds, s.win_lds());
    }
    // the work list: problem after problem, each problem's units longest
    // first and the problems in order of their longest unit, so the launch
    // starts with the longest units, keeps one or two problems' FSR data in
    // the caches at a time, and ends with short units
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    auto head = [&](int i) {
        const std::vector<float> &c = active[i]->solver.work_cost;
        return c.empty() ? 0.f : c[0];
    };
    // problems whose groups fit one lane (G <= 8) first: they run in their
    // own launch with the one-chunk lane layout
    auto one_chunk = [&](int i) { return active[i]->solver.info.n_groups <= kGL; };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        if (one_chunk(x) != one_chunk(y)) return one_chunk(x);
        if (small(x) != small(y)) return small(x);
        return head(x) > head(y);
    });
    std::vector<int> us2, uc2;
    int n_c1 = 0, n_small = 0;
    for (int i : order) {
        const std::vector<int> &w = active[i]->solver.work_host;
        us2.insert(us2.end(), w.size(), i);
        uc2.insert(uc2.end(), w.begin(), w.end());
        if (one_chunk(i)) n_c1 += (int)w.size();
        if (small(i)) n_small += (int)w.size();
    }
    if (!us2.empty()) {
        SRV_HIPCHK(hipMemcpyAsync(d_uslot, us2.data(), us2.size() * 4, hipMemcpyHostToDevice, stream));
        SRV_HIPCHK(hipMemcpyAsync(d_ucode, uc2.data(), uc2.size() * 4, hipMemcpyHostToDevice, stream));
    }
    SRV_HIPCHK(hipMemcpyAsync(d_blk, blk.data(), (n + 1) * 4, hipMemcpyHostToDevice, stream));
    // descriptors and FSR tables stay fixed while the batch does; each
    // problem's iteration count (its boundary-buffer parity) and stopping
    // state are kept on the device and advanced by the step itself
    for (int i = 0; i < n; ++i) {
        const Request *r = active[i];
        h_win[i] = r->solver.win_args_batched();
        if (small(i)) h_win[i].Sw = r->solver.lane_sw;
        h_fsr[i] = r->solver.fsr_args();
        h_ctl[i] = SlotCtl{r->opts.tol, r->opts.max_iters, r->iters, 0, 0};
    }
    if (n > 0) {
        SRV_HIPCHK(hipMemcpyAsync(d_win, h_win, n * sizeof(WinArgs), hipMemcpyHostToDevice, stream));
        SRV_HIPCHK(hipMemcpyAsync(d_fsr, h_fsr, n * sizeof(FsrArgs), hipMemcpyHostToDevice, stream));
        SRV_HIPCHK(hipMemcpyAsync(d_ctl, h_ctl, n * sizeof(SlotCtl), hipMemcpyHostToDevice, stream));
    }
    SRV_HIPCHK(hipStreamSynchronize(stream));
    batch.win_table = d_win;
    batch.fsr_table = d_fsr;
    batch.blk_pre = d_blk;
    batch.u_slot = d_uslot;
    batch.u_code = d_ucode;
    batch.res_dev = d_res;
    batch.ctl = d_ctl;
    batch.n_slots = n;
    batch.n_units = (int)us2.size();
    batch.n_units_c1 = n_c1;
    batch.n_units_small = n_small;
    batch.fsr_blocks = blk[n];
    batch.lds = lds;
    batch.lds_small = lds_small;
    for (int b = 0; b < 2; ++b) {
        if (exec[b]) {
            (void)hipGraphExecDestroy(exec[b]);
            exec[b] = nullptr;
        }
        if (graph[b]) {
            (void)hipGraphDestroy(graph[b]);
            graph[b] = nullptr;
        }
    }
    if (stream && n > 0) {
        // one step = batched iteration, residuals to one half of the pinned buffer
        for (int b = 0; b < 2; ++b) {
            SRV_HIPCHK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
            const int rc = launch_batch_step(batch, stream);
            hipError_t e = hipSuccess;
            if (!rc) e = hipMemcpyAsync(h_res + (size_t)b * max_slots, d_res, n * 8, hipMemcpyDeviceToHost, stream);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(stream, &g);
            if (e != hipSuccess || rc || e2 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                set_error("graph capture of the batched step failed");
                return MOC_EDEVICE;
            }
            graph[b] = g;
            SRV_HIPCHK(hipGraphInstantiate(&exec[b], graph[b], nullptr, nullptr, 0));
        }
    }
    dirty = false;
    return MOC_OK;
}

void Server::retire(Request *r) {
    r->solver.read_stats(&r->stats);
    r->stats.iters = r->iters;
    r->stats.residual = r->residual;
    r->state = DONE;
}

// Launch one batched step whose residuals land in the given half.
int Server::launch(int half) {
    const int n = (int)active.size();
    if (exec[half]) {
        SRV_HIPCHK(hipGraphLaunch(exec[half], stream));
    } else {
        const int rc = launch_batch_step(batch, stream);
        if (rc) return rc;
        SRV_HIPCHK(hipMemcpyAsync(h_res + (size_t)half * max_slots, d_res, n * 8, hipMemcpyDeviceToHost, stream));
    }
    SRV_HIPCHK(hipEventRecord(done_ev[half], stream));
    return MOC_OK;
}

// Wait for the step of one half and account it: every running problem has
// done one more iteration.  The stopping rule is the device's (the same
// inputs, so the same decision): an iteration after the first whose residual
// is < tol, or max_iters.  A stopped problem is skipped by the steps still in
// flight and retires at the next drain.
int Server::collect(int half, bool *changed) {
    SRV_HIPCHK(hipEventSynchronize(done_ev[half]));
    const double *res = h_res + (size_t)half * max_slots;
    for (size_t i = 0; i < active.size(); ++i) {
        Request *r = active[i];
        if (r->stopped) continue;
        ++r->solver.iter;
        ++r->iters;
        r->residual = r->iters <= 1 ? 1.0 : res[i];
        const bool conv = r->iters > 1 && r->residual < r->opts.tol;
        if (conv || r->iters >= r->opts.max_iters) {
            r->converged = conv;
            r->stopped = true;
            *changed = true;
        }
    }
    return MOC_OK;
}

// One server step.  With nothing in flight: admit, rebuild if the batch
// changed, launch.  Then the next step is launched before the current one is
// read, so the GPU does not wait for the host between steps; problems that
// stop are skipped by the device from then on, so running ahead changes no
// result.  The pipeline drains (and stopped requests retire) when a problem
// stops or a queued request could be admitted.
int Server::step(int *n_active, int *n_queued) {
    int rc = MOC_OK;
    if (inflight < 0) {
        rc = admit();
        if (rc) return rc;
        if (dirty) {
            rc = rebuild();
            if (rc) return rc;
        }
        if (!active.empty()) {
            rc = launch(next_half);
            if (rc) return rc;
            inflight = next_half;
            next_half ^= 1;
        }
    }
    if (inflight >= 0) {
        rc = launch(next_half);
        if (rc) return rc;
        const int second = next_half;
        next_half ^= 1;
        bool changed = false;
        rc = collect(inflight, &changed);
        if (rc) return rc;
        if (changed || admissible()) {
            rc = collect(second, &changed);
            if (rc) return rc;
            inflight = -1;
            std::vector<Request *> keep;
            for (Request *r : active) {
                if (r->stopped) retire(r);
                else keep.push_back(r);
            }
            if (keep.size() != active.size()) dirty = true;
            active.swap(keep);
        } else {
            inflight = second;
        }
    }
    if (n_active) *n_active = (int)active.size();
    if (n_queued) *n_queued = (int)queue.size();
    return MOC_OK;
}

}  // namespace moc

struct moc_server {
    moc::Server s;
};

using moc::set_error;

extern "C" {

static size_t server_table_bytes(int max_slots) {
    return moc::align_up(max_slots * sizeof(moc::WinArgs)) + moc::align_up(max_slots * sizeof(moc::FsrArgs)) +
           moc::align_up((max_slots + 1) * 4) + 2 * moc::align_up(moc::kUnitCap * 4) +
           moc::align_up(max_slots * 8) + moc::align_up(max_slots * sizeof(moc::SlotCtl));
}

int moc_server_arena_overhead(int max_slots, size_t *bytes) {
    if (!bytes || max_slots < 1 || max_slots > 4096) {
        set_error("need bytes != NULL and 1 <= max_slots <= 4096");
        return MOC_EINVAL;
    }
    *bytes = server_table_bytes(max_slots);
    return MOC_OK;
}

int moc_server_create(void *dev_arena, size_t arena_bytes, int max_slots, void *stream,
                      moc_server **out) {
    if (!out) {
        set_error("out is NULL");
        return MOC_EINVAL;
    }
    *out = nullptr;
    if (!dev_arena || max_slots < 1 || max_slots > 4096) {
        set_error("need a device arena and 1 <= max_slots <= 4096");
        return MOC_EINVAL;
    }
    if ((reinterpret_cast<uintptr_t>(dev_arena) & (moc::kAlign - 1)) != 0) {
        set_error("arena must be 256-byte aligned");
        return MOC_EINVAL;
    }
    moc_server *sv = new (std::nothrow) moc_server();
    if (!sv) {
        set_error("host allocation failed");
        return MOC_ENOMEM;
    }
    moc::Server &s = sv->s;
    s.arena = static_cast<char *>(dev_arena);
    s.arena_bytes = arena_bytes;
    {
        // default fill target: 64 work units per compute unit (two resident
        // sweep workgroups per CU, 32 rounds of them)
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            s.fill_units = 64LL * cus;
    }
    s.max_slots = max_slots;
    s.stream = static_cast<hipStream_t>(stream);
    // device tables at the front of the arena
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off += moc::align_up(b);
        return o;
    };
    const size_t o_win = take(max_slots * sizeof(moc::WinArgs));
    const size_t o_fsr = take(max_slots * sizeof(moc::FsrArgs));
    const size_t o_blk = take((max_slots + 1) * 4);
    const size_t o_us = take(moc::kUnitCap * 4);
    const size_t o_uc = take(moc::kUnitCap * 4);
    const size_t o_res = take(max_slots * 8);
    const size_t o_ctl = take(max_slots * sizeof(moc::SlotCtl));
    if (off >= arena_bytes) {
        delete sv;
        set_error("arena too small for the server tables");
        return MOC_ENOMEM;
    }
    s.d_win = reinterpret_cast<moc::WinArgs *>(s.arena + o_win);
    s.d_fsr = reinterpret_cast<moc::FsrArgs *>(s.arena + o_fsr);
    s.d_blk = reinterpret_cast<int *>(s.arena + o_blk);
    s.d_uslot = reinterpret_cast<int *>(s.arena + o_us);
    s.d_ucode = reinterpret_cast<int *>(s.arena + o_uc);
    s.d_res = reinterpret_cast<double *>(s.arena + o_res);
    s.d_ctl = reinterpret_cast<moc::SlotCtl *>(s.arena + o_ctl);
    if (off != server_table_bytes(max_slots)) {
        delete sv;
        set_error("internal: server table size mismatch");
        return MOC_EINVAL;
    }
    s.usable_bytes = arena_bytes - off;
    s.alloc.init(off, s.usable_bytes);
    if (hipHostMalloc((void **)&s.h_win, max_slots * sizeof(moc::WinArgs), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&s.h_fsr, max_slots * sizeof(moc::FsrArgs), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&s.h_ctl, max_slots * sizeof(moc::SlotCtl), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&s.h_res, 2 * max_slots * 8, hipHostMallocDefault) != hipSuccess) {
        delete sv;
        set_error("pinned host allocation failed");
        return MOC_ENOMEM;
    }
    for (int b = 0; b < 2; ++b)
        if (hipEventCreateWithFlags(&s.done_ev[b], hipEventDisableTiming) != hipSuccess) {
            delete sv;
            set_error("event creation failed");
            return MOC_EDEVICE;
        }
    *out = sv;
    return MOC_OK;
}

void moc_server_destroy(moc_server *srv) {
    if (!srv) return;
    (void)hipStreamSynchronize(srv->s.stream);
    delete srv;
}

int moc_server_submit(moc_server *srv, const moc_plan *plan, const double *q,
                      const moc_solve_opts *opts, unsigned long long *ticket) {
    if (!srv || !plan || !q || !opts || !ticket) {
        set_error("NULL argument");
        return MOC_EINVAL;
    }
    if (opts->max_iters < 1 || !(opts->tol >= 0) || opts->sweep_fp64 || opts->exp_mode) {
        set_error("serving runs the FP32 sweep with the stable exponential; need max_iters >= 1, tol >= 0");
        return MOC_EINVAL;
    }
    moc::Server &s = srv->s;
    const moc::Plan &p = plan->p;
    const moc_plan_info inf = p.info();
    if (moc::window_fit(p, false) < 1) {
        set_error("plan not servable: one 2D segment x layers x groups exceeds the LDS window");
        return MOC_EINVAL;
    }
    auto r = std::make_unique<moc::Request>();
    r->ticket = s.next_ticket++;
    r->plan = std::make_unique<moc::Plan>(p);
    const size_t nq = (size_t)inf.n_fsr * inf.n_groups;
    for (size_t i = 0; i < nq; ++i)
        if (!(q[i] >= 0) || !std::isfinite(q[i])) {
            set_error("source must be finite and >= 0");
            return MOC_EINVAL;
        }
    r->q.assign(q, q + nq);
    r->opts = *opts;
    r->bytes = inf.workspace_bytes;
    r->units = 2 * inf.n_2d_tracks;
    if (moc::align_up(r->bytes) > s.usable_bytes || r->units > (long long)moc::kUnitCap) {
        set_error("request can never fit the arena");
        return MOC_ENOMEM;
    }
    *ticket = r->ticket;
    s.queue.push_back(r.get());
    s.all[r->ticket] = std::move(r);
    return MOC_OK;
}

int moc_server_step(moc_server *srv, int *n_active, int *n_queued) {
    if (!srv) {
        set_error("NULL server");
        return MOC_EINVAL;
    }
    return srv->s.step(n_active, n_queued);
}

int moc_server_set_fill(moc_server *srv, long long max_units) {
    if (!srv || max_units < 0) {
        set_error("need a server and max_units >= 0");
        return MOC_EINVAL;
    }
    srv->s.fill_units = max_units;
    return MOC_OK;
}

int moc_server_query(const moc_server *srv, unsigned long long ticket, int *done) {
    if (!srv || !done) {
        set_error("NULL argument");
        return MOC_EINVAL;
    }
    auto it = srv->s.all.find(ticket);
    if (it == srv->s.all.end()) {
        set_error("unknown ticket");
        return MOC_EINVAL;
    }
    *done = it->second->state == moc::DONE ? 1 : 0;
    return MOC_OK;
}

int moc_server_poll(moc_server *srv, unsigned long long ticket, moc_stats *stats,
                    double *flux_out, size_t n) {
    if (!srv) {
        set_error("NULL server");
        return MOC_EINVAL;
    }
    moc::Server &s = srv->s;
    auto it = s.all.find(ticket);
    if (it == s.all.end()) {
        set_error("unknown ticket");
        return MOC_EINVAL;
    }
    moc::Request &r = *it->second;
    if (r.state != moc::DONE) return MOC_EBUSY;
    const size_t nfg = (size_t)r.solver.info.n_fsr * r.solver.info.n_groups;
    if (flux_out) {
        if (n != nfg) {
            set_error("flux size must be n_fsr * n_groups");
            return MOC_EINVAL;
        }
        hipError_t e = hipMemcpyAsync(flux_out, r.solver.ws + r.solver.lay.off_phi, nfg * 8,
                                      hipMemcpyDeviceToHost, s.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
        if (e != hipSuccess) {
            set_error(hipGetErrorString(e));
            return MOC_EDEVICE;
        }
    }
    if (stats) *stats = r.stats;
    const bool conv = r.converged;
    s.alloc.release(r.off, r.bytes);
    s.all.erase(it);
    return conv ? MOC_OK : MOC_ENOTCONV;
}

}  // extern "C"
