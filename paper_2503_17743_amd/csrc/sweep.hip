// gfx950 kernels of one fixed-source 3D MOC source iteration:
//   source update -> on-the-fly 3D segment generation + Eq. 3 sweep + FSR
//   tally + boundary angular-flux exchange -> finalize (Eq. 4 estimator,
//   residual, balance).
//
// Sweep mapping.  One wavefront (64 lanes) takes a bundle of T consecutive
// lines of one z-stack (paper Eq. 5: same 2D track, same polar angle, dz
// apart) in one sweep direction.  Lane = (line in bundle, group chunk): the G
// groups are split into C = ceil(G/8) chunks across lanes and each lane keeps
// the angular flux of its chunk's (at most 8) groups in registers, so T =
// 64/C lines (64 for G <= 8).  All lines of a bundle project onto the same 2D
// track, so the wave walks that track's 2D segments in lockstep (uniform loop,
// the segment record is shared by the whole wave) and every lane splits the
// current 2D segment at the axial planes its line crosses (Eqs. 6-11
// evaluated per line: a line inside one layer over the whole 2D segment has
// length ds/sin(theta) (Eq. 8), a line crossing a whole layer has length
// dz_layer/|cos(theta)| (Eq. 11)); the piece geometry is computed once per
// line and reused for all groups of the lane.  3D segments live only in
// registers: nothing per 3D track or segment is stored.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "args.hpp"
#include "plan.hpp"
#include "solver.hpp"

namespace moc {

constexpr double kFourPi = 12.566370614359172953850573533118;
// dynamic LDS per windowed-sweep workgroup: 64 KB, or up to 78 KB (still two
// workgroups per CU) when 64 KB holds only a few 2D segments of all layers
constexpr size_t kWinLdsBudget = 64 * 1024;
constexpr size_t kWinLdsBudgetDeep = 78 * 1024;
constexpr int kWinDeepBelow = 8;
// Per-lane walk on shallow stacks: 256-thread workgroups with 40 KB windows
// (four per CU), used when such a window still holds kWinSmallMinSw segments
constexpr size_t kWinLdsBudgetSmall = 40 * 1024;
constexpr int kWinSmallMinSw = 16;
// Per-lane walk on deep stacks: 1024-thread workgroups (one per CU, the same
// 16 waves per CU) with windows of up to 156 KB, used when the 512-thread
// window holds fewer than kWinBigBelow segments and the large one at least
// twice as many: fewer windows per line, so fewer carries of a line's flux
// between windows and fewer per-line set-ups
constexpr int kWinThreadsBig = 1024;
constexpr size_t kWinLdsBudgetBig = 156 * 1024;
constexpr int kWinBigBelow = 16;
constexpr int kSlots = 64;        // spread of the scalar accumulators
constexpr size_t kScalBytes = 128 * 1024;   // scalar block of a workspace
constexpr int kSlotStride = 16;   // doubles between slots (separate cache lines)

// scalar accumulator layout inside the scalar block (doubles / u64)
enum ScalarQ { Q_SIN = 0, Q_SOUT, Q_LEAK, Q_NSEG, Q_LINKERR, Q_BAL, Q_ABS, Q_SRC, Q_RES,
               Q_PNEW, Q_POLD, Q_SHAPE, Q_COUNT };
static_assert(64 + (size_t)Q_COUNT * 64 * 16 <= kScalBytes / 8, "scalar slots exceed the scalar block");
__host__ __device__ inline size_t slot_index(int q, int slot) {
    return 64 + ((size_t)q * kSlots + slot) * kSlotStride;
}

// ------------------------------------------------------------------ helpers

constexpr float kLog2e = 1.44269504088896341f;
// F = 1 - 2^{-u} at u = s l (the attenuation factor 1 - e^{-tau} of Eq. 3,
// with s = Sigma_t log2(e) and l the piece length), without cancellation,
// from one hardware exp2 and one hardware log2.  With e = 2^{-u'}(1 + d) the
// value the exp2 returns for u' = s l rounded, 1 - e is exact for e >= 1/2
// but off by e d, which for small u is most of F.  log2 e = -u' + d/ln 2 up
// to the log2's own error, about one ulp of its result (also for e near 1,
// where that result is small), so du = s l + log2 e (one rounding) =
// (s l - u') + d/ln 2, and F = (1 - e) + ln 2 e du = 1 - 2^{-s l} + O(d^2):
// the correction also takes back the rounding of s l.  The product e du is
// a legacy multiply (0 x anything = 0), so that where e underflows to 0 and
// log2 e is -inf, F comes out as 1.  Measured on the device over every float
// u in [2^-30, 256] (s = 1): within 1.71 ulp of FP64.  Split in two so that
// a caller evaluating several groups can issue all its exp2 first.
__device__ inline float atten_e(float s, float l) { return __builtin_amdgcn_exp2f(-(s * l)); }
__device__ inline float atten_from_e(float s, float l, float e) {
    const float du = fmaf(s, l, __builtin_amdgcn_logf(e));
    float m;
    asm("v_mul_legacy_f32 %0, %1, %2" : "=v"(m) : "v"(e), "v"(du));
    return fmaf(0.693147182f, m, 1.0f - e);
}
__device__ inline float atten_f32(float s, float l) { return atten_from_e(s, l, atten_e(s, l)); }

// F(tau) = 1 - e^{-tau} for tau >= 0 (the same evaluation, s = log2(e))
__device__ inline float one_minus_exp_f32(float t) { return atten_f32(kLog2e, t); }

template <typename R>
__device__ inline R one_minus_exp(R tau, int exp_mode);

template <>
__device__ inline float one_minus_exp<float>(float tau, int exp_mode) {
    if (exp_mode == 0) return one_minus_exp_f32(tau);
    return 1.0f - __expf(-tau);      // naive form, precision study only
}
template <>
__device__ inline double one_minus_exp<double>(double tau, int) {
    return -expm1(-tau);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline long long wave_sum_ll(long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// 2D-length interval [ls, le] of the line z = base + c l inside the box
// (0 <= l <= Lt, 0 <= z <= H); ic = 1/c
__device__ inline void clip_line(double base, double c, double ic, double Lt, double H, double &ls,
                                 double &le) {
    double a, b;
    if (c > 0) {
        a = -base * ic;
        b = (H - base) * ic;
    } else {
        a = (H - base) * ic;
        b = -base * ic;
    }
    ls = a > 0 ? a : 0.0;
    le = b < Lt ? b : Lt;
}

// largest k in [lo, hi) with pos[k] <= x (pos[lo] == 0 <= x assumed)
__device__ inline int seg_search(const double *__restrict__ pos, int lo, int hi, double x) {
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (pos[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}


// z of line i of stack s at the start of its 2D track (Eq. 5)
__device__ inline double line_base(const SweepArgs &a, long long s, long long i) {
    return a.zeta[s] + (double)(a.ilo[s] + i) * a.dz;
}

// Incremental walk of one line through its 2D segments in sweep order.  The
// line z = base + c l crosses the axial plane z = m h at l = m h/c - base/c;
// between two consecutive crossings it stays in one layer, so a 2D segment
// [s0, s1] splits into pieces at the crossings that fall inside it (Eqs. 6-7
// locate them per FSR; here per line).  Each piece has 3D length
// dl / sin(theta): a whole 2D segment inside one layer gives Eq. 8, a whole
// layer crossed gives h / |cos(theta)| (Eq. 11).  Crossing positions are
// evaluated directly, never accumulated, so no rounding drifts along a line.
struct Walker {
    double lcur;    // current 2D position
    double lnp;     // 2D position of the next plane crossing in sweep order
    double hc, bc;  // h / c and base / c
    int k;          // current layer
    int mnext;      // index of the next plane
    int kstep;      // +1 moving up, -1 moving down
};

__device__ inline void walk_init(Walker &w, double base, double c, double ic, double h, double inv_h,
                                 int K, double l0, bool bwd) {
    const bool up = (c > 0) != bwd;
    const double z0 = base + c * l0;
    int k = up ? (int)floor(z0 * inv_h) : (int)ceil(z0 * inv_h) - 1;
    k = min(max(k, 0), K - 1);
    w.k = k;
    w.kstep = up ? 1 : -1;
    w.mnext = up ? k + 1 : k;
    w.hc = h * ic;
    w.bc = base * ic;
    w.lcur = l0;
    w.lnp = w.mnext * w.hc - w.bc;
}

// Walk from the current position to e (the end of this 2D segment in sweep
// order) and call f(layer, length, valid) for every piece; valid is false for
// pieces shorter than kMinSeg (the caller adds nothing for them).  Returns
// the number of valid pieces.
template <bool BWD, typename F>
__device__ __forceinline__ int walk_segment(Walker &w, double e, double secl, int K, F &&f) {
    int m = 0;
    for (;;) {
        const bool cross = BWD ? (w.lnp > e) : (w.lnp < e);
        const double lend = cross ? w.lnp : e;
        const double l3 = (BWD ? (w.lcur - lend) : (lend - w.lcur)) * secl;
        const bool valid = l3 >= kMinSeg;
        f(min(max(w.k, 0), K - 1), l3, valid);
        m += valid;
        w.lcur = lend;
        if (!cross) break;
        w.k += w.kstep;
        w.mnext += w.kstep;
        w.lnp = w.mnext * w.hc - w.bc;
    }
    return m;
}

// Where a directed line meets the box boundary at its start (at_exit false)
// or end (at_exit true) in sweep order: kind 0 = a z face (at 2D position lz),
// 1 = the side face at the 2D track end, 2 = the edge where both meet.
struct Bound {
    int kind;
    int face_z, face_s;
    double lz, zf, lside;
};

__device__ inline Bound boundary_of(double base, double c, double ic, double Lt, double H, int dir,
                                    bool at_exit, int meta) {
    Bound b;
    const bool up = (c > 0) != (dir == 1);
    const bool top = at_exit ? up : !up;
    b.zf = top ? H : 0.0;
    b.face_z = top ? MOC_FACE_ZMAX : MOC_FACE_ZMIN;
    b.lz = (b.zf - base) * ic;
    const bool far_end = (dir == 0) == at_exit;     // the l = Lt end of the 2D track
    b.lside = far_end ? Lt : 0.0;
    b.face_s = far_end ? ((meta >> 20) & 0xf) : ((meta >> 16) & 0xf);
    if (far_end) b.kind = (b.lz < Lt - kTrackEps) ? 0 : (b.lz > Lt + kTrackEps) ? 1 : 2;
    else b.kind = (b.lz > kTrackEps) ? 0 : (b.lz < -kTrackEps) ? 1 : 2;
    return b;
}

__device__ inline bool is_vacuum(const SweepArgs &a, const Bound &b) {
    return (b.kind != 1 && a.bc[b.face_z] == MOC_BC_VACUUM) ||
           (b.kind != 0 && a.bc[b.face_s] == MOC_BC_VACUUM);
}

// Directed slot (2 * stored track + dir) of the track that continues a line
// leaving through reflective boundary b: specular reflection on a z face keeps
// the 2D track and mirrors the polar angle; on a side face the 2D successor is
// taken from the cyclic links; through an edge both apply.  The line index on
// the successor's z-stack follows from matching z at the shared point (Eq. 5).
// Returns -1 if no such line exists.
__device__ inline long long successor_line(const SweepArgs &a, const Bound &b, long long t, int n,
                                           int dir, double base, double c, int &n2, long long &i2);
__device__ inline long long successor_slot(const SweepArgs &a, const Bound &b, long long t, int n,
                                           int dir, double base, double c) {
    int n2;
    long long i2;
    return successor_line(a, b, t, n, dir, base, c, n2, i2);
}

// The same, also giving the continuation's polar index n2 and line index i2
// in its stack.
__device__ inline long long successor_line(const SweepArgs &a, const Bound &b, long long t, int n,
                                           int dir, double base, double c, int &n2, long long &i2) {
    long long t2;
    int d2;
    double l2, z2;
    const int P = a.P;
    if (b.kind == 0) {
        t2 = t;
        d2 = dir;
        n2 = P - 1 - n;
        l2 = b.lz;
        z2 = b.zf;
    } else {
        const int lk = a.t_link[2 * t + dir];
        t2 = lk >> 1;
        d2 = lk & 1;
        const bool same = (d2 == dir);
        n2 = ((b.kind == 1) == same) ? n : P - 1 - n;
        l2 = d2 == 0 ? 0.0 : a.t_len[t2];
        z2 = b.kind == 1 ? base + c * b.lside : b.zf;
    }
    const long long s2 = t2 * P + n2;
    const double c2 = a.cot[(a.t_meta[t2] & 0xffff) * P + n2];
    i2 = llrint((z2 - a.zeta[s2] - c2 * l2) * a.inv_dz) - a.ilo[s2];
    if (i2 < 0 || i2 >= (long long)a.cnt[s2]) return -1;
    return 2 * (a.trk_off[s2] + i2) + d2;
}

// ------------------------------------------------------------------ direct sweep
// One wave = one work item (2*chunk + dir): a bundle of T consecutive lines of
// one z-stack, lane = (line, group chunk), every 3D segment-group tallied with
// one FP64 global atomic.  Used when an LDS window of one 2D segment x all
// layers x all groups does not fit (very large K*G).
template <typename R, typename B>
__global__ __launch_bounds__(256) void k_sweep(SweepArgs a) {
    const int lane = threadIdx.x & 63;
    const long long w = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (w >= a.n_items) return;
    const long long item = a.items ? a.items[w] : w;
    const int dir = (int)(item & 1);
    const long long chunk = item >> 1;
    long long lo = 0, hi = a.n_stacks;
    while (hi - lo > 1) {
        long long mid = (lo + hi) >> 1;
        if (a.chunk_off[mid] <= chunk) lo = mid;
        else hi = mid;
    }
    const long long s = lo;
    const int P = a.P, G = a.G, K = a.K, C = a.C, GL = a.GL;
    const long long t = s / P;
    const int n = (int)(s - t * P);
    const int meta = a.t_meta[t];
    const int an = (meta & 0xffff) * P + n;
    const double c = a.cot[an], ic = a.icot[an], secl = a.secl[an], W = a.wgt[an];
    const double Lt = a.t_len[t];
    const int f0 = a.t_first[t], f1 = a.t_first[t + 1];
    const int tr = lane / C;
    const int g0 = (lane - tr * C) * GL;
    const int ng = max(0, min(GL, G - g0));
    const long long zi = (chunk - a.chunk_off[s]) * a.T + tr;
    const bool active = (tr < a.T) && (zi < (long long)a.cnt[s]) && ng > 0;
    const double base = line_base(a, s, zi);
    double ls = 1e300, le = -1e300;
    if (active) clip_line(base, c, ic, Lt, a.H, ls, le);
    const double l_lo = wave_min(ls), l_hi = wave_max(le);
    const long long slot_in = 2 * (a.trk_off[s] + zi) + dir;
    const R *sigt = (const R *)a.sigt;
    const R *qhat = (const R *)a.qhat;
    const size_t hook = (size_t)w * kItemStride + (size_t)tr * G + g0;
    R psi[kGL];
#pragma unroll
    for (int j = 0; j < kGL; ++j) psi[j] = 0;
    double s_in = 0.0;
    if (active && a.mode == 0) {
        const bool from_vacuum = is_vacuum(a, boundary_of(base, c, ic, Lt, a.H, dir, false, meta));
#pragma unroll
        for (int j = 0; j < kGL; ++j)
            if (j < ng) {
                if (a.psi_entry) psi[j] = (R)a.psi_entry[hook + j];
                else if (!from_vacuum) psi[j] = (R)((const B *)a.psi_in)[slot_in * G + g0 + j];
                s_in += W * (double)psi[j];
            }
    }
    long long nseg = 0;
    const int k_first = seg_search(a.seg_pos, f0, f1, l_lo);
    const int k_last = seg_search(a.seg_pos, f0, f1, l_hi);
    Walker wk;
    if (active) walk_init(wk, base, c, ic, a.h, a.inv_h, K, dir ? le : ls, dir == 1);
    const int nk = k_last - k_first + 1;
    for (int kk = 0; kk < nk; ++kk) {
        const int k = dir ? (k_last - kk) : (k_first + kk);
        const double s0 = a.seg_pos[k];
        const double s1 = (k + 1 < f1) ? a.seg_pos[k + 1] : Lt;
        const int reg = a.seg_reg[k];
        if (!active) continue;
        const double e = dir ? fmax(s0, ls) : fmin(s1, le);
        if (!(dir ? e < wk.lcur : e > wk.lcur)) continue;
        const long long jb = (long long)reg * K;
        const R *st = sigt + a.reg_mat[reg] * G + g0;
        auto piece = [&](int kz, double l3, bool valid) {
            if (!valid) return;
            const long long j0 = (jb + kz) * G + g0;
            if (a.mode == 1) {
                if (g0 == 0) unsafeAtomicAdd(&a.acc[jb + kz], W * l3 / kFourPi);
                return;
            }
#pragma unroll
            for (int j = 0; j < kGL; ++j)
                if (j < ng) {
                    const R d = (psi[j] - qhat[j0 + j]) * one_minus_exp<R>(st[j] * (R)l3, a.exp_mode);
                    psi[j] -= d;                                                   // Eq. 3
                    unsafeAtomicAdd(&a.acc[j0 + j], W * (double)d);
                }
        };
        nseg += dir ? walk_segment<true>(wk, e, secl, K, piece) : walk_segment<false>(wk, e, secl, K, piece);
    }
    if (a.mode == 1) {
        const long long tot = wave_sum_ll(active && g0 == 0 ? nseg : 0);
        if (lane == 0)
            atomicAdd((unsigned long long *)&a.scal[slot_index(Q_NSEG, (int)(w % kSlots))],
                      (unsigned long long)tot);
        return;
    }
    double leak = 0.0, s_out = 0.0;
    long long link_err = 0;
    if (active) {
        double wpsi = 0.0;
#pragma unroll
        for (int j = 0; j < kGL; ++j)
            if (j < ng) {
                wpsi += W * (double)psi[j];
                if (a.psi_exit) a.psi_exit[hook + j] = (double)psi[j];
            }
        s_out = wpsi;
        const Bound b = boundary_of(base, c, ic, Lt, a.H, dir, true, meta);
        if (is_vacuum(a, b)) {
            leak = wpsi;
        } else if (a.psi_out) {
            const long long slot2 = successor_slot(a, b, t, n, dir, base, c);
            if (slot2 >= 0) {
#pragma unroll
                for (int j = 0; j < kGL; ++j)
                    if (j < ng) ((B *)a.psi_out)[slot2 * G + g0 + j] = (B)psi[j];
            } else {
                link_err = 1;
                leak = wpsi;
            }
        }
    }
    const double v_in = wave_sum(s_in), v_out = wave_sum(s_out), v_lk = wave_sum(leak);
    const long long ns = wave_sum_ll(active ? nseg * ng : 0);
    const long long le_ = wave_sum_ll(link_err);
    if (lane == 0) {
        const int sl = (int)(w % kSlots);
        unsafeAtomicAdd(&a.scal[slot_index(Q_SIN, sl)], v_in);
        unsafeAtomicAdd(&a.scal[slot_index(Q_SOUT, sl)], v_out);
        unsafeAtomicAdd(&a.scal[slot_index(Q_LEAK, sl)], v_lk);
        atomicAdd((unsigned long long *)&a.scal[slot_index(Q_NSEG, sl)], (unsigned long long)ns);
        if (le_) atomicAdd((unsigned long long *)&a.scal[slot_index(Q_LINKERR, sl)], (unsigned long long)le_);
    }
}

// ------------------------------------------------------------------ windowed sweep
// One workgroup = one 2D track in one sweep direction (every polar stack,
// every line).  The track's 2D segments are walked in windows of Sw segments.
// For each window the reduced source of all Sw x K x G FSR-groups the window
// can touch is staged in LDS (for a segment they are contiguous: FSRs
// r*K .. r*K+K-1, layer-fastest) and an FP64 LDS tally of the same shape
// collects W * delta_psi from every line of every polar stack that crosses
// the window; the tally is then added to HBM with one atomic per touched
// FSR-group.  Waves take bundles of T consecutive lines of one stack (lane =
// line x group chunk) and walk the window's segments in lockstep.  A line's angular
// flux is carried from window to window in its own boundary slot (read once
// at its start, then free); a line starting on a vacuum face starts from 0.
constexpr int kWinThreads = 512;
constexpr int kWinWaves = kWinThreads / 64;
constexpr int kMaxPolar = 64;
constexpr size_t kWinFixedLds = 2048;   // per-stack line ranges and bundle prefix

// Byte offset of the FP64 tally: after the reduced source, 8-byte aligned.
__host__ __device__ inline size_t win_acc_offset(int Sw, int KG, int rbytes) {
    return ((size_t)Sw * KG * rbytes + 7) & ~(size_t)7;
}

// Dynamic LDS of a window of Sw segments (layout in sweep_unit).
__host__ __device__ inline size_t win_lds_bytes(int Sw, int K, int G, int rbytes) {
    const size_t kg = (size_t)K * G;
    return win_acc_offset(Sw, (int)kg, rbytes) + (size_t)Sw * kg * 8 + ((size_t)Sw + 1) * 8 +
           (size_t)Sw * G * rbytes + (size_t)Sw * 2 * 4 + kWinFixedLds;
}


// floor(a / b) for 0 <= a < 2^20 and 1 <= b: the float estimate a * (1/b)
// (hardware reciprocal) is within one of the quotient, and one correction
// step in integers makes it exact
__device__ inline int div_small(int a, int b) {
    int q = (int)((float)a * __builtin_amdgcn_rcpf((float)b));
    const int r = a - q * b;
    q += (r >= b) ? 1 : 0;
    q -= (r < 0) ? 1 : 0;
    return q;
}

__device__ inline int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Wait until this wave's vector memory operations have completed, among them
// global_load_lds writes into LDS, which the compiler does not track
// (s_waitcnt vmcnt(0); the expcnt and lgkmcnt fields left at their maximum)
__device__ inline void wait_lds_loads() { __builtin_amdgcn_s_waitcnt(0x0F70); }
__device__ inline float uniform_val(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ inline double uniform_val(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// MODE 0: transport sweep; MODE 1: volume tally (W l / 4 pi per FSR).
// EXPM 0: stable 1 - e^-tau; EXPM 1: 1 - hardware exp (precision study).
// GC > 0: the group count is the compile-time constant GC (with C1), so the
// per-group loops are straight-line code; GC = 0: G from the arguments.
// LANE (MODE 0, C1): every lane takes one piece of its own line per step and
// moves on to its next 2D segment by itself (reading that segment's Sigma_t
// row from LDS), instead of the whole wave taking every 2D segment together.
// Both walks give every line the same pieces in the same order.
// EXP (per-lane walk only): 0 on-the-fly sweep; 1 store pass of the
// stored-segment sweep (wa.exp_pass: 1 count the wave steps and bundle windows
// of each unit, 2 write each bundle window's step count to the step table,
// 3 record every lane's pieces), which walks the geometry only; 2 replay: the
// transport sweep reads the recorded pieces instead of walking the geometry.
template <typename R, typename B, int MODE, int EXPM, bool BWD, bool C1, int GC = 0, bool LANE = false,
          int NT = kWinThreads, int EXP = 0>
__device__ __forceinline__ void sweep_unit(const WinArgs &wa, int code, int unit,
                                           unsigned char *smem, bool flip = false,
                                           const ChainItem *ci = nullptr) {
    static_assert(!LANE || (MODE == 0 && C1), "the per-lane walk is the one-chunk transport sweep");
    static_assert(EXP == 0 || LANE, "the stored-segment sweep records the per-lane walk");
    // the transport arithmetic runs in the on-the-fly sweep and in the replay
    constexpr bool kPhys = EXP != 1;
    const SweepArgs &a = wa.s;
    // boundary buffers of this sweep (flip: the descriptor's pair swapped)
    void *const psi_in = flip ? a.psi_out : a.psi_in;
    void *const psi_out = flip ? a.psi_in : a.psi_out;
    const int tid = threadIdx.x, lane = tid & 63, wave = uniform(tid >> 6);
    const int G = GC > 0 ? GC : a.G, K = a.K, P = a.P, T = a.T;
    // most lines of one stack a bundle may skip (the lines per axial layer)
    const int Smax = wa.lstride;
    // C1: all groups of a line in one lane (G <= kGL), the common case
    const int C = C1 ? 1 : a.C, GL = C1 ? G : a.GL;
    const int KG = K * G;
    const int Sw = wa.Sw;
    // LDS: [reduced source Sw*KG | FP64 tally Sw*KG | segment starts Sw+1 |
    //       Sigma_t Sw*G | regions 2*Sw | line ranges].  The reduced source sits
    // at offset 0, so a lane's per-group loads address it with immediate
    // offsets from one register.
    R *q_l = (R *)smem;
    double *acc_l = (double *)(smem + win_acc_offset(Sw, KG, (int)sizeof(R)));
    double *s_pos = acc_l + (size_t)Sw * KG;
    R *s_st = (R *)(s_pos + Sw + 1);
    int *s_reg = (int *)(s_st + (size_t)Sw * G);      // two buffers of Sw
    int *r_lo = s_reg + 2 * Sw;
    int *r_hi = r_lo + kMaxPolar;
    int *r_st = r_hi + kMaxPolar;       // line stride of each stack's bundles
    int *bpre = r_st + kMaxPolar;
    // per-lane walk: complete blocks of each stack's bundles, and the lines
    // per bundle (q or q + 1, the first x bundles longer) of its last block
    int *r_full = bpre + kMaxPolar + 1;
    int *r_q = r_full + kMaxPolar;
    int *r_x = r_q + kMaxPolar;
    int *s_next = r_x + kMaxPolar;      // next bundle of the window to take
    // FP32 stable attenuation: Sigma_t is staged times log2(e), so that
    // Sigma_t l is the exponent of 2 itself
    constexpr bool kL2 = std::is_same<R, float>::value && EXPM == 0 && MODE == 0;

    const long long t = code >> 1;
    constexpr int dir = BWD ? 1 : 0;
    const int meta = a.t_meta[t];
    const int az = meta & 0xffff;
    const double Lt = a.t_len[t];
    const int f0 = a.t_first[t], f1 = a.t_first[t + 1];
    const int nwin = (f1 - f0 + Sw - 1) / Sw;
    const int fn = wa.filt_n ? wa.filt_n[unit] : -1;
    const long long fi0 = wa.filt_i0 ? wa.filt_i0[unit] : 0;
    const R *sigt = (const R *)a.sigt;
    const R *qhat = (const R *)a.qhat;
    // lane = (line tr of the bundle, group chunk): groups g0 .. g0+ng-1
    const int tr = C == 1 ? lane : lane / C;
    const int g0 = (lane - tr * C) * GL;
    const int ng = max(0, min(GL, G - g0));

    for (int i = tid; i < Sw * KG; i += NT) acc_l[i] = 0.0;

    double s_in = 0.0, s_out = 0.0, leak = 0.0;
    // pieces of this lane (a 32-bit count: a lane takes far fewer than 2^31
    // pieces in one unit), widened for the wave total
    int nseg = 0;
    long long link_err = 0;
    // stored-segment sweep: step-table entry of the current window's first
    // bundle (every bundle window of the unit in sweep order), and the count
    // pass's totals of this wave
    unsigned bw_run = (EXP != 0 && wa.exp_tbase) ? wa.exp_tbase[unit] : 0u;
    unsigned long long exp_steps = 0;

    // Staging of a window: segment starts, regions, Sigma_t and the reduced
    // source of every FSR-group the window can touch.  Window wi + 1 is
    // staged during window wi's tally flush, into areas the flush does not
    // read (the regions, which it reads, are double-buffered).  The reduced
    // source goes straight from HBM to LDS (global_load_lds: a wave fills 64
    // consecutive entries, each lane gathering its own), so its loads hold no
    // registers and their latency overlaps the flush; the few other values
    // are loaded before the flush and written after it.  The caller waits for
    // the LDS loads (wait_lds_loads) before the barrier that publishes them.
    auto window_of = [&](const int wi, int &k0, int &nsw) {
        const int w = dir ? nwin - 1 - wi : wi;
        k0 = f0 + w * Sw;
        nsw = min(k0 + Sw, f1) - k0;
    };
    // flush of window wi's tally: one HBM atomic per touched FSR-group (the
    // volume tally has one entry per FSR, kept in the g = 0 slots)
    auto flush_window = [&](const int wi) {
        int k0, nsw;
        window_of(wi, k0, nsw);
        const int *reg_of = s_reg + (wi & 1) * Sw;
        for (int i = tid; i < nsw * KG && kPhys; i += NT) {
            const double v = acc_l[i];
            if (v != 0.0) {
                const int kk = i / KG;
                const int rem = i - kk * KG;
                const size_t reg = (size_t)reg_of[kk];
                if (MODE == 0) unsafeAtomicAdd(&a.acc[reg * KG + rem], v);
                else unsafeAtomicAdd(&a.acc[reg * K + rem / G], v);
                acc_l[i] = 0.0;
            }
        }
    };
    const int n_srch = lane;
    const bool srch = wave == 0 && n_srch < P && (fn < 0 || fn == n_srch);
    // Chain sweep: the lines of this stack the item sweeps, those that
    // entered the box (rising: through the bottom face, falling: the top one)
    // within [A, B) of the traversal: segment seg of nseg, its bounds whole
    // numbers of the stack's entry spacing lc / kk (kk lines cross a point per
    // cycle).  A line at z (at H - z when falling) where this unit starts
    // entered a 2D distance z / |cot| earlier, at the unrolled position
    // u - z / |cot|.  The bounds fall half a spacing from every entry point
    // (the traversals start where all lines sit at (i + 1/2) dz), so the
    // closed forms need no check.
    int ch_lo = 0, ch_hi = 0x7fffffff;
    if (ci && srch) {
        const long long s = t * P + n_srch;
        const double c = a.cot[az * P + n_srch];
        const double ce = dir ? -c : c;
        const double z0 = a.zeta[s] + (double)a.ilo[s] * a.dz + c * (dir ? Lt : 0.0);
        const double kk = rint(ci->lc * fabs(c) * a.inv_dz);
        const double sp = ci->lc / kk;
        const double ea = floor((double)ci->seg * kk / (double)ci->nseg) * sp;
        const double eb = floor((double)(ci->seg + 1) * kk / (double)ci->nseg) * sp;
        // entry distance d in (x0, x1]
        const double x0 = ci->u - eb, x1 = ci->u - ea;
        const double cnt_s = (double)a.cnt[s];
        double flo, fhi;
        if (ce > 0) {
            flo = floor((ce * x0 - z0) * a.inv_dz) + 1.0;
            fhi = floor((ce * x1 - z0) * a.inv_dz);
        } else {
            flo = ceil((a.H + ce * x1 - z0) * a.inv_dz);
            fhi = ceil((a.H + ce * x0 - z0) * a.inv_dz) - 1.0;
        }
        ch_lo = (int)fmin(fmax(flo, 0.0), cnt_s);
        ch_hi = (int)fmin(fmax(fhi, -1.0), cnt_s - 1.0);
    }
    auto search_window = [&](const int wi) {
        int k0, nsw;
        window_of(wi, k0, nsw);
        const double wa_ = a.seg_pos[k0];
        const double wb_ = (k0 + nsw < f1) ? a.seg_pos[k0 + nsw] : Lt;
        int cs = 0;
        double c_s = 0.0, ic_s = 0.0, zeta_s = 0.0;
        long long ilo_s = 0;
        if (srch) {
            const long long s = t * P + n_srch;
            cs = a.cnt[s];
            c_s = a.cot[az * P + n_srch];
            ic_s = a.icot[az * P + n_srch];
            zeta_s = a.zeta[s];
            ilo_s = a.ilo[s];
        }
        if (tid == 0) *s_next = NT / 64;
        int lo = 0, hi = -1;
        if (srch) {
            const double c = c_s, ic = ic_s;
            // z of line i at the track start: the value line_base gives
            auto base_of = [&](int i) { return zeta_s + (double)(ilo_s + i) * a.dz; };
            auto ls_lt = [&](int i) {
                double l0, l1;
                clip_line(base_of(i), c, ic, Lt, a.H, l0, l1);
                return l0 < wb_;
            };
            auto le_gt = [&](int i) {
                double l0, l1;
                clip_line(base_of(i), c, ic, Lt, a.H, l0, l1);
                return l1 > wa_;
            };
            // The line bases are evenly spaced, so the two ends have closed
            // forms (for c > 0 a line starts before wb when base > -wb c and
            // ends after wa when base < H - wa c; for c < 0 the same with wa
            // and wb exchanged).  Each estimate is accepted only when the
            // exact predicate confirms it at the estimate and its neighbour,
            // else found by bisection, so the result is the bisection's.
            auto rising = [&](int i) { return c > 0 ? ls_lt(i) : le_gt(i); };    // false ... true
            auto falling = [&](int i) { return c > 0 ? le_gt(i) : ls_lt(i); };   // true ... false
            const double z0 = zeta_s + (double)ilo_s * a.dz;
            const double z_lo = c > 0 ? -wb_ * c : -wa_ * c, z_hi = c > 0 ? a.H - wa_ * c : a.H - wb_ * c;
            int a0 = (int)fmin(fmax(floor((z_lo - z0) * a.inv_dz) + 1.0, 0.0), (double)cs);
            int b0 = (int)fmin(fmax(ceil((z_hi - z0) * a.inv_dz) - 1.0, -1.0), (double)cs - 1.0);
            // first true of the rising predicate in [0, cs] (cs: none)
            if (!((a0 == cs || rising(a0)) && (a0 == 0 || !rising(a0 - 1)))) {
                int a1 = cs;
                a0 = 0;
                while (a0 < a1) { int m = (a0 + a1) >> 1; if (rising(m)) a1 = m; else a0 = m + 1; }
            }
            // last true of the falling predicate in [-1, cs - 1] (-1: none)
            if (!((b0 == -1 || falling(b0)) && (b0 == cs - 1 || !falling(b0 + 1)))) {
                int b1 = cs - 1;
                b0 = -1;
                while (b0 < b1) { int m = (b0 + b1 + 1) >> 1; if (falling(m)) b0 = m; else b1 = m - 1; }
            }
            lo = a0;
            hi = b0;
            if (ci) {
                lo = max(lo, ch_lo);
                hi = min(hi, ch_hi);
            }
            if (fn >= 0) {
                lo = max(lo, (int)fi0);
                hi = min(hi, (int)fi0 + T - 1);
            }
        }
        // bundles: blocks of S*T consecutive lines, each split into S
        // bundles of every S-th line.  Lanes S lines (S dz) apart fall in
        // different layers, so fewer lanes of one instruction add to the
        // same LDS tally entry.  S = ceil(lines / T), at most the lines
        // per layer, keeps the bundle count of consecutive bundles.
        // The per-lane walk packs the lines of all stacks into bundles
        // instead (the prefix then counts lines): lanes need no common
        // polar angle there, and the stacks' partial bundles merge.
        int nb = 0, S = 1, full = 0, q = 0, x = 0;
        if (hi >= lo) {
            const int nl = hi - lo + 1;
            S = min(Smax, (nl + T - 1) / T);
            const int ST = S * T;
            const int blocks = (nl + ST - 1) / ST;
            nb = LANE ? nl : (blocks - 1) * S + min(S, nl - (blocks - 1) * ST);
            full = (nl - 1) / ST;
            const int rem = nl - full * ST;
            q = rem / S;
            x = rem - q * S;
        }
        int sc = nb;
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(sc, o, 64);
            if (lane >= o) sc += v;
        }
        r_lo[lane] = lo;
        r_hi[lane] = hi;
        r_st[lane] = S;
        bpre[lane + 1] = sc;
        if (lane == 0) bpre[0] = 0;
        if (LANE) {
            r_full[lane] = full;
            r_q[lane] = q;
            r_x[lane] = x;
        }
    };
    // n dwords from HBM straight into LDS (global_load_lds: chunk c of 64
    // dwords by wave c mod waves, each lane copying one; the reduced source
    // below moves 16 B per lane, the LDS taking lane L's at 16 L); the caller waits
    // for them (wait_lds_loads) before the barrier that publishes them
    auto copy_to_lds = [&](void *dst, const void *src, const int n) {
        for (int c = wave; c * 64 < n; c += NT / 64) {
            const int i = c * 64 + lane;
            if (i < n)
                __builtin_amdgcn_global_load_lds(
                    (const __attribute__((address_space(1))) void *)((const unsigned *)src + i),
                    (__attribute__((address_space(3))) void *)((unsigned *)dst + c * 64), 4, 0, 0);
        }
    };
    // stage window wi; with prev >= 0, flush window prev between the loads
    // and the writes
    auto stage_window = [&](const int wi, const int prev) {
        int k0, nsw;
        window_of(wi, k0, nsw);
        // FP32 sweep: segment starts, regions and Sigma_t rows are copies of
        // contiguous HBM ranges, and the reduced source a gather by region,
        // all loaded straight into LDS; the FP64 sweep and the naive-exp
        // study load into registers and write after the flush
        constexpr bool kDirect = sizeof(R) == 4;
        int *reg_to = s_reg + (wi & 1) * Sw;
        if constexpr (kDirect) {
            copy_to_lds(s_pos, a.seg_pos + k0, 2 * nsw);
            copy_to_lds(reg_to, a.seg_reg + k0, nsw);
            if (MODE == 0 && kPhys) {
                if (kL2) copy_to_lds(s_st, a.seg_st + (size_t)k0 * G, nsw * G);
                // reduced source: entry i of segment kk = i / KG, from the
                // region lane kk of every wave holds for windows of up to 64
                // segments (waiting for it here keeps every wait out of the
                // loop), else read per entry.  The window fits the LDS, so
                // nsw * KG is far below 2^20 (the range of div_small).
                const int nq = nsw * KG;
                const bool lane_regs = nsw <= 64;
                int reg_lane = 0;
                if (lane_regs) {
                    reg_lane = lane < nsw ? a.seg_reg[k0 + lane] : 0;
                    wait_lds_loads();
                }
                if (KG % 4 == 0) {
                    // 16 B per lane (four entries of one row: rows and the
                    // workspace are 16-byte aligned), a quarter of the loads
                    for (int c = wave; c * 256 < nq; c += NT / 64) {
                        const int i = c * 256 + 4 * lane;
                        const int kk = div_small(min(i, nq - 4), KG);
                        int r = __shfl(reg_lane, kk & 63, 64);
                        if (!lane_regs) r = a.seg_reg[k0 + kk];
                        if (i < nq)
                            __builtin_amdgcn_global_load_lds(
                                (const __attribute__((address_space(1))) void *)(qhat + (size_t)r * KG + (i - kk * KG)),
                                (__attribute__((address_space(3))) void *)(q_l + c * 256), 16, 0, 0);
                    }
                } else {
                    for (int c = wave; c * 64 < nq; c += NT / 64) {
                        const int i = c * 64 + lane;
                        const int kk = div_small(min(i, nq - 1), KG);
                        int r = __shfl(reg_lane, kk & 63, 64);
                        if (!lane_regs) r = a.seg_reg[k0 + kk];
                        if (i < nq)
                            __builtin_amdgcn_global_load_lds(
                                (const __attribute__((address_space(1))) void *)(qhat + (size_t)r * KG + (i - kk * KG)),
                                (__attribute__((address_space(3))) void *)(q_l + c * 64), 4, 0, 0);
                    }
                }
            }
        }
        const double wb = (k0 + nsw < f1) ? a.seg_pos[k0 + nsw] : Lt;
        double pos = 0.0;
        int reg = 0;
        if (!kDirect && tid < nsw) {
            pos = a.seg_pos[k0 + tid];
            reg = a.seg_reg[k0 + tid];
        }
        constexpr bool kStRegs = !(kDirect && kL2);
        R st = (R)0;
        if (MODE == 0 && kPhys && kStRegs && tid < nsw * G) {
            const int kk = tid / G;
            const int m = a.reg_mat[a.seg_reg[k0 + kk]] * G + (tid - kk * G);
            st = kL2 ? (R)(a.sigt64[m] * 1.4426950408889634) : sigt[m];
        }
        if (wave == 0) search_window(wi);
        if (prev >= 0) flush_window(prev);
        if constexpr (!kDirect) {
            if (tid < nsw) {
                s_pos[tid] = pos;
                reg_to[tid] = reg;
            }
            for (int i = tid + NT; i < nsw; i += NT) {
                s_pos[i] = a.seg_pos[k0 + i];
                reg_to[i] = a.seg_reg[k0 + i];
            }
        }
        if (tid == 0) s_pos[nsw] = wb;
        if (MODE == 0 && kPhys && sizeof(R) == 8) {
            for (int i = tid; i < nsw * KG; i += NT) {
                const int kk = i / KG;
                q_l[i] = qhat[(size_t)a.seg_reg[k0 + kk] * KG + (i - kk * KG)];
            }
        }
        if (MODE == 0 && kPhys && kStRegs) {
            if (tid < nsw * G) s_st[tid] = st;
            for (int i = tid + NT; i < nsw * G; i += NT) {
                const int kk = i / G;
                const int m = a.reg_mat[a.seg_reg[k0 + kk]] * G + (i - kk * G);
                s_st[i] = kL2 ? (R)(a.sigt64[m] * 1.4426950408889634) : sigt[m];
            }
        }
    };
    if (nwin > 0) stage_window(0, -1);
    wait_lds_loads();
    __syncthreads();

    for (int wi = 0; wi < nwin; ++wi) {
        int k0, nsw;
        window_of(wi, k0, nsw);
        const double wa_ = s_pos[0];
        const double wb_ = s_pos[nsw];
        const int n_lines = bpre[P];     // per-lane walk: lines of all stacks
        const int total = LANE ? (n_lines + T - 1) / T : bpre[P];
        // bundles: wave w takes w, w + waves, ...; or, with wa.dyn_bundles,
        // its first one so and then the next untaken one (an LDS counter)
        // whenever it finishes one, so that the waves end the window together
        auto next_bundle = [&](int cur) -> int {
            if (!wa.dyn_bundles) return cur + NT / 64;
            int v = 0;
            if (lane == 0) v = atomicAdd(s_next, 1);
            return uniform(__shfl(v, 0, 64));
        };
        for (int bnd = wave; bnd < total; bnd = next_bundle(bnd)) {
            int n = 0, i = 0, nact = 0;
            bool active;
            if constexpr (LANE) {
                // entry g of the window's packed list: stack n, and its line
                // in the order of the strided bundles above (those bundles
                // concatenated), so neighbouring lanes stay S lines apart
                // (T = 64 lines per bundle here: one chunk of groups per lane)
                const int g = bnd * 64 + tr;
                const int gg = min(g, n_lines - 1);
                while (bpre[n + 1] <= gg) ++n;
                const int lo = r_lo[n], S = r_st[n];
                const int ST = S * 64, full = r_full[n];        // complete blocks
                const int p = gg - bpre[n];
                const int b = min(div_small(p, ST), full);
                const int within = p - b * ST;
                int r, k;
                if (b < full) {
                    r = within >> 6;
                    k = within & 63;
                } else {
                    // last block: its lines in min(S, lines) bundles of q or
                    // q + 1 lines, the first x of them one line longer
                    const int q = r_q[n], x = r_x[n];
                    if (within < x * (q + 1)) {
                        r = div_small(within, q + 1);
                        k = within - r * (q + 1);
                    } else {
                        const int w2 = within - x * (q + 1);
                        const int r2 = div_small(w2, q);
                        r = x + r2;
                        k = w2 - r2 * q;
                    }
                }
                i = lo + b * ST + r + S * k;
                active = g < n_lines && tr < T && ng > 0;
            } else {
                while (bpre[n + 1] <= bnd) ++n;
                n = uniform(n);
                const int bl = bnd - bpre[n];
                const int S = uniform(r_st[n]);
                const int i0 = uniform(r_lo[n] + (bl / S) * S * T + bl % S);
                nact = uniform(min(T, (r_hi[n] - i0) / S + 1));    // lines in this bundle (>= 1)
                i = i0 + S * tr;
                active = (tr < nact) && ng > 0;
            }
            const long long s = t * P + n;
            const int an = az * P + n;
            const double c = a.cot[an], ic = a.icot[an], secl = a.secl[an], W = a.wgt[an];
            const double base = line_base(a, s, i);
            double ls = 1e300, le = -1e300;
            if (active) clip_line(base, c, ic, Lt, a.H, ls, le);
            // segments of the window the bundle can touch, [ka, kb]: with the
            // per-lane walk the whole window (each lane finds its own first
            // segment and stops where its line ends, so a narrower range
            // would change no piece and only cost two wave reductions and
            // two bisections per bundle); with the lockstep walk the range
            // the bundle's lines span, which the wave walks together
            int ka = 0, kb = nsw - 1;
            if constexpr (!LANE) {
                // the extents of consecutive lines of one stack move
                // monotonically with the line index, so the first and last
                // line bound them
                const int last = (nact - 1) * C;
                const double u_lo = fmax(fmin(__shfl(ls, 0, 64), __shfl(ls, last, 64)), wa_);
                const double u_hi = fmin(fmax(__shfl(le, 0, 64), __shfl(le, last, 64)), wb_);
                int lo2 = 0, hi2 = nsw;
                while (hi2 - lo2 > 1) { const int m = (lo2 + hi2) >> 1; if (s_pos[m] <= u_lo) lo2 = m; else hi2 = m; }
                ka = lo2;
                lo2 = ka;
                hi2 = nsw;
                while (hi2 - lo2 > 1) { const int m = (lo2 + hi2) >> 1; if (s_pos[m] < u_hi) lo2 = m; else hi2 = m; }
                kb = lo2;
                // the same for every lane (the bounds came through lane shuffles)
                ka = uniform(ka);
                kb = uniform(kb);
            }
            const bool starts = dir == 0 ? (ls >= wa_) : (le <= wb_);
            const bool ends = dir == 0 ? (le <= wb_) : (ls >= wa_);
            // the line's flux between windows (and on entry): its boundary
            // slot, or in the chain sweep its entry of the item's carry
            // buffer (parity, stack, line)
            const long long slot = ci ? ((long long)n * ci->cap + i) : 2 * (a.trk_off[s] + i) + dir;
            B *const cbuf = ci ? (B *)ci->cur : (B *)psi_in;
            const size_t hook = (size_t)unit * kItemStride + (size_t)(i - fi0) * G + g0;
            R psi[kGL];
#pragma unroll
            for (int j = 0; j < kGL; ++j) psi[j] = 0;
            // the lane carries W * psi along its line: then W * delta_psi is
            // what Eq. 3 yields directly, and the tally needs no multiply
            const R Wr = (R)W;
            if (MODE == 0 && kPhys && active) {
                const B *pin = cbuf + slot * G + g0;
                if (!starts) {
                    // carried from the previous window (already scaled by W)
#pragma unroll
                    for (int j = 0; j < kGL; ++j)
                        if (j < ng) psi[j] = (R)pin[j];
                } else {
                    const bool from_vacuum =
                        !a.psi_entry && is_vacuum(a, boundary_of(base, c, ic, Lt, a.H, dir, false, meta));
#pragma unroll
                    for (int j = 0; j < kGL; ++j)
                        if (j < ng) {
                            if (a.psi_entry) psi[j] = (R)a.psi_entry[hook + j];
                            else if (!from_vacuum) psi[j] = (R)pin[j];
                            s_in += W * (double)psi[j];
                            psi[j] *= Wr;
                        }
                }
            }
            Walker wk;
            if (active) walk_init(wk, base, c, ic, a.h, a.inv_h, K, dir ? fmin(le, wb_) : fmax(ls, wa_), dir == 1);
            // a piece's tally atomics are issued after the next piece's reduced
            // source loads, so those loads do not wait behind them (LDS
            // operations of a wave complete in order)
            R pend[kGL];
            int pend_li = -1;
            auto flush_pending = [&]() {
                if (MODE == 0 && pend_li >= 0) {
#pragma unroll
                    for (int j = 0; j < kGL; ++j)
                        if (j < GL)
                            __hip_atomic_fetch_add(&acc_l[pend_li + (C1 ? j : min(j, ng - 1))], (double)pend[j],
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            };
            // Eq. 3 on one piece for the lane's groups (one-chunk lanes, C1):
            // d = W (psi - qhat) F(Sigma_t l); with the FP32 exp2 form, all
            // groups' exp2 are issued first, so that no transcendental waits on
            // the one just issued (the per-lane walk and its replay share this,
            // so both give the same fluxes bit for bit)
            auto transport = [&](const R (&qv)[kGL], const R (&stv)[kGL], const R lr) {
                if constexpr (kL2) {
                    float e[kGL];
#pragma unroll
                    for (int j = 0; j < kGL; ++j)
                        if (j < GL) e[j] = atten_e((float)stv[j], (float)lr);
#pragma unroll
                    for (int j = 0; j < kGL; ++j)
                        if (j < GL) {
                            const R f = (R)atten_from_e((float)stv[j], (float)lr, e[j]);
                            const R d = fma(-Wr, qv[j], psi[j]) * f;
                            psi[j] -= d;
                            pend[j] = d;
                        }
                } else {
#pragma unroll
                    for (int j = 0; j < kGL; ++j)
                        if (j < GL) {
                            const R f = one_minus_exp<R>(stv[j] * lr, EXPM);
                            const R d = fma(-Wr, qv[j], psi[j]) * f;
                            psi[j] -= d;
                            pend[j] = d;
                        }
                }
            };
            if constexpr (LANE && EXP == 2) {
                // replay of the recorded pieces of this bundle window: the
                // same transport arithmetic as the per-lane walk below, with
                // each step's piece read instead of generated
                const unsigned off = wa.exp_table[bw_run + bnd];
                const int nst = (int)(wa.exp_table[bw_run + bnd + 1] - off);
                const Piece *src = wa.exp_data + (size_t)off * 64 + lane;
                // the pieces of the next kReplayAhead steps are in flight while
                // this step computes (HBM latency spans several steps)
                constexpr int kReplayAhead = 4;
                const Piece none{0u, -1.0f};
                Piece ahead[kReplayAhead];
#pragma unroll
                for (int d = 0; d < kReplayAhead; ++d) ahead[d] = d < nst ? src[(size_t)d * 64] : none;
                for (int step = 0; step < nst; ++step) {
                    const Piece cur = ahead[0];
#pragma unroll
                    for (int d = 0; d + 1 < kReplayAhead; ++d) ahead[d] = ahead[d + 1];
                    ahead[kReplayAhead - 1] =
                        step + kReplayAhead < nst ? src[(size_t)(step + kReplayAhead) * 64] : none;
                    if (cur.len >= 0.0f) {
                        const int li = (int)(cur.idx & 0xffffu);
                        const int lst = (int)__umul24(cur.idx >> 16, (unsigned)G);
                        const R lr = (R)cur.len;
                        R qv[kGL], stv[kGL];
#pragma unroll
                        for (int j = 0; j < kGL; ++j)
                            if (j < GL) {
                                qv[j] = q_l[li + j];
                                stv[j] = s_st[lst + j];
                            }
                        flush_pending();
                        transport(qv, stv, lr);
                        pend_li = li;
                        nseg += cur.len > 0.0f;
                    }
                }
            } else if constexpr (LANE) {
                // the lane's first 2D segment: the one holding its start in
                // sweep order (inside the window, since its extent is)
                const int kstep = dir ? -1 : 1;
                int sg = dir ? kb : ka;
                double e = 0.0;
                bool fin = !active;
                if (active) {
                    const double l0 = wk.lcur;
                    int lo2 = ka, hi2 = kb + 1;
                    while (hi2 - lo2 > 1) {
                        const int m = (lo2 + hi2) >> 1;
                        if (dir ? (s_pos[m] < l0) : (s_pos[m] <= l0)) lo2 = m;
                        else hi2 = m;
                    }
                    sg = lo2;
                    e = dir ? fmax(s_pos[sg], ls) : fmin(s_pos[sg + 1], le);
                }
                // each lane walks its own segments, reading its segment's
                // Sigma_t row from LDS; LDS indices of the lane's segment:
                // tally / reduced source row and Sigma_t row
                int lq = sg * KG + g0, lst = sg * G;
                // every step takes a piece of at least one lane, and a line has
                // at most (segments) + K + 2 pieces in the window: a bound on
                // the steps that the walk never reaches
                const int max_steps = 64 * (kb - ka + 1 + K + 2) + 8;
                // store pass: this bundle window's first recorded wave step
                const unsigned rec_off = (EXP == 1 && wa.exp_pass == 3) ? wa.exp_table[bw_run + bnd] : 0u;
                int steps_done = 0;
                for (int step = 0; step < max_steps; ++step) {
                    if (__ballot(!fin) == 0) break;
                    ++steps_done;
                    Piece rec{0u, -1.0f};
                    if (!fin) {
                        const bool cross = dir ? (wk.lnp > e) : (wk.lnp < e);
                        const double lend = cross ? wk.lnp : e;
                        const double l3 = (dir ? (wk.lcur - lend) : (lend - wk.lcur)) * secl;
                        const bool valid = l3 >= kMinSeg;
                        const int kz = min(max(wk.k, 0), K - 1);
                        const int li = lq + (int)__umul24((unsigned)kz, (unsigned)G);
                        const R lr = valid ? (R)l3 : (R)0;
                        if constexpr (EXP == 1) {
                            rec.idx = (unsigned)li | ((unsigned)sg << 16);
                            rec.len = (float)lr;
                        } else {
                        R qv[kGL], stv[kGL];
#pragma unroll
                        for (int j = 0; j < kGL; ++j)
                            if (j < GL) {
                                qv[j] = q_l[li + j];
                                stv[j] = s_st[lst + j];
                            }
                        flush_pending();
                        transport(qv, stv, lr);
                        pend_li = li;
                        }
                        nseg += valid;
                        wk.lcur = lend;
                        if (cross) {
                            wk.k += wk.kstep;
                            wk.mnext += wk.kstep;
                            wk.lnp = wk.mnext * wk.hc - wk.bc;
                        } else if (sg == (dir ? ka : kb) || e == (dir ? ls : le)) {
                            fin = true;      // the line leaves the bundle's segments here
                        } else {
                            sg += kstep;
                            lq += kstep * KG;
                            lst += kstep * G;
                            const double sp = s_pos[dir ? sg : sg + 1];
                            e = dir ? (sp > ls ? sp : ls) : (sp < le ? sp : le);
                        }
                    }
                    if constexpr (EXP == 1)
                        if (wa.exp_pass == 3) wa.exp_data[((size_t)rec_off + step) * 64 + lane] = rec;
                }
                if constexpr (EXP == 1) {
                    if (wa.exp_pass == 2 && lane == 0) wa.exp_table[bw_run + bnd] = (unsigned)steps_done;
                    exp_steps += (unsigned long long)steps_done;
                }
            } else {
            const int nk = kb - ka + 1;
            for (int q = 0; q < nk; ++q) {
                const int kk = dir ? (kb - q) : (ka + q);
                const double s0 = s_pos[kk], s1 = s_pos[kk + 1];
                if (!active) continue;
                const double e = dir ? fmax(s0, ls) : fmin(s1, le);
                if (!(dir ? e < wk.lcur : e > wk.lcur)) continue;
                const int lb = kk * KG + g0;
                if (MODE == 1) {
                    nseg += walk_segment<BWD>(wk, e, secl, K, [&](int kz, double l3, bool valid) {
                        if (g0 == 0 && valid)
                            __hip_atomic_fetch_add(&acc_l[lb + kz * G], W * l3 / kFourPi, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                    });
                    continue;
                }
                // Sigma_t of the segment's material for the lane's groups (the
                // same for every lane when C1: held in scalar registers).  The
                // group loop bound GL is uniform; a lane of the last chunk with
                // fewer groups repeats its last group with a zero update.
                R stv[kGL];
#pragma unroll
                for (int j = 0; j < kGL; ++j)
                    if (j < GL) stv[j] = C1 ? uniform_val(s_st[kk * G + j]) : s_st[kk * G + g0 + min(j, ng - 1)];
                nseg += walk_segment<BWD>(wk, e, secl, K, [&](int kz, double l3, bool valid) {
                    const int li = lb + (int)__umul24((unsigned)kz, (unsigned)G);
                    // a piece below kMinSeg adds nothing: F(0) = 0 keeps psi unchanged
                    const R lr = valid ? (R)l3 : (R)0;
                    R qv[kGL];
#pragma unroll
                    for (int j = 0; j < kGL; ++j)
                        if (j < GL) qv[j] = q_l[li + (C1 ? j : min(j, ng - 1))];
                    flush_pending();
#pragma unroll
                    for (int j = 0; j < kGL; ++j)
                        if (j < GL) {
                            // d = W (psi - qhat) (1 - e^-tau)  (Eq. 3 on the scaled flux)
                            const R f = kL2 ? (R)atten_f32((float)stv[j], (float)lr)
                                            : one_minus_exp<R>(stv[j] * lr, EXPM);
                            R d = fma(-Wr, qv[j], psi[j]) * f;
                            if (!C1 && j >= ng) d = (R)0;
                            psi[j] -= d;
                            pend[j] = d;
                        }
                    pend_li = li;
                });
            }
            }
            flush_pending();
            if (MODE == 0 && kPhys && active) {
                if (!ends) {
                    B *pc = cbuf + slot * G + g0;                   // carried to the next window
#pragma unroll
                    for (int j = 0; j < kGL; ++j)
                        if (j < ng) pc[j] = (B)psi[j];
                } else {
                    // back to the angular flux itself at the line's end
                    const R iW = (R)(1.0 / W);
                    double wpsi = 0.0;
#pragma unroll
                    for (int j = 0; j < kGL; ++j)
                        if (j < ng) {
                            wpsi += (double)psi[j];
                            psi[j] *= iW;
                            if (a.psi_exit) a.psi_exit[hook + j] = (double)psi[j];
                        }
                    s_out += wpsi;
                    const Bound b = boundary_of(base, c, ic, Lt, a.H, dir, true, meta);
                    if (is_vacuum(a, b)) {
                        leak += wpsi;
                    } else if (psi_out || ci) {
                        int n2;
                        long long i2;
                        long long slot2 = successor_line(a, b, t, n, dir, base, c, n2, i2);
                        // chain sweep: the continuation is swept by the next
                        // item, from the other carry buffer
                        if (ci && slot2 >= 0) slot2 = (long long)n2 * ci->cap + i2;
                        if (slot2 >= 0) {
                            B *po = (ci ? (B *)ci->next : (B *)psi_out) + slot2 * G + g0;
#pragma unroll
                            for (int j = 0; j < kGL; ++j)
                                if (j < ng) po[j] = (B)psi[j];
                        } else {
                            ++link_err;
                            leak += wpsi;
                        }
                    }
                }
            }
        }
        __syncthreads();
        if constexpr (EXP == 1)
            if (wa.exp_pass == 1 && tid == 0) atomicAdd(&wa.exp_count[2 * (size_t)unit + 1], (unsigned long long)total);
        bw_run += (unsigned)total;
        // the window's tally to HBM, and the next window staged meanwhile
        if (wi + 1 < nwin) stage_window(wi + 1, wi);
        else flush_window(wi);
        wait_lds_loads();
        __syncthreads();
    }
    if constexpr (EXP == 1) {
        // store pass: the count pass adds this wave's steps to its unit
        if (wa.exp_pass == 1 && lane == 0) atomicAdd(&wa.exp_count[2 * (size_t)unit], exp_steps);
        return;
    }
    // per-wave totals -> spread scalar slots
    const double v_in = wave_sum(s_in), v_out = wave_sum(s_out), v_lk = wave_sum(leak);
    const long long ns = wave_sum_ll(MODE == 1 ? (g0 == 0 ? (long long)nseg : 0) : (long long)nseg * ng);
    const long long le_ = wave_sum_ll(link_err);
    if (lane == 0) {
        const int sl = (int)(((long long)unit * (NT / 64) + wave) % kSlots);
        if (MODE == 0) {
            unsafeAtomicAdd(&a.scal[slot_index(Q_SIN, sl)], v_in);
            unsafeAtomicAdd(&a.scal[slot_index(Q_SOUT, sl)], v_out);
            unsafeAtomicAdd(&a.scal[slot_index(Q_LEAK, sl)], v_lk);
            if (le_) atomicAdd((unsigned long long *)&a.scal[slot_index(Q_LINKERR, sl)], (unsigned long long)le_);
        }
        atomicAdd((unsigned long long *)&a.scal[slot_index(Q_NSEG, sl)], (unsigned long long)ns);
    }
}

// FP32 arithmetic: capped at 128 VGPRs so that two 512-thread workgroups
// share a CU (4 waves per SIMD).  C1: G <= 8, all groups of a line in one lane.
template <typename B, int MODE, int EXPM, bool C1, int GC = 0>
__global__ __launch_bounds__(kWinThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_sweep_win(WinArgs wa) {
    extern __shared__ __align__(16) unsigned char smem[];
    // the direction is uniform per workgroup: specialise the whole unit on it
    const int code = wa.work[blockIdx.x];
    if (code & 1) sweep_unit<float, B, MODE, EXPM, true, C1, GC>(wa, code, blockIdx.x, smem);
    else sweep_unit<float, B, MODE, EXPM, false, C1, GC>(wa, code, blockIdx.x, smem);
}

// The FP32 transport sweep with the per-lane walk (one-chunk lanes, G = GC).
// NT threads per workgroup (512, or 256 with the shorter windows of shallow
// stacks: fewer waves wait at each window's barrier).  EXP 0: the on-the-fly
// sweep; EXP 2: the replay of recorded pieces (stored-segment sweep).  With
// wa.persist_units > 0 the grid is persistent: workgroup b sweeps the units
// b, b + gridDim.x, ... of the work list (a static assignment, as in a
// grid-stride loop over tracks); otherwise one workgroup per unit.
template <typename B, int GC, int NT, int EXP = 0, bool PERSIST = false>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_sweep_win_lane(WinArgs wa) {
    extern __shared__ __align__(16) unsigned char smem[];
    if constexpr (PERSIST) {
        for (int u = blockIdx.x; u < wa.persist_units; u += gridDim.x) {
            const int code = wa.work[u];
            if (code & 1) sweep_unit<float, B, 0, 0, true, true, GC, true, NT, EXP>(wa, code, u, smem);
            else sweep_unit<float, B, 0, 0, false, true, GC, true, NT, EXP>(wa, code, u, smem);
        }
    } else {
        const int code = wa.work[blockIdx.x];
        if (code & 1) sweep_unit<float, B, 0, 0, true, true, GC, true, NT, EXP>(wa, code, blockIdx.x, smem);
        else sweep_unit<float, B, 0, 0, false, true, GC, true, NT, EXP>(wa, code, blockIdx.x, smem);
    }
}

// Chain-line sweep (vacuum top and bottom faces): each workgroup takes the
// next segment of a traversal (a directed 2D cycle) from a counter and
// sweeps its items, the units its lines cross, in traversal order.  The
// flux a line leaves through a side face goes to its continuation's entry
// of the workgroup's other carry buffer, which the next item (the next unit)
// reads, so every line is swept whole within the sweep (no flux lags an
// iteration) and no boundary buffer is needed.  A segment's first unit holds
// the entry points of its first lines, so no flux enters it from an earlier
// item; the segments are independent.
template <typename B, int GC, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_sweep_win_chain(WinArgs wa) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_seg;
    ChainItem ci;
    ci.cap = wa.chain_cap;
    const size_t cstride = (size_t)wa.s.P * wa.chain_cap * wa.s.G;
    B *const carry = (B *)wa.chain_carry + (size_t)blockIdx.x * 2 * cstride;
    for (;;) {
        if (threadIdx.x == 0) s_seg = (int)atomicAdd(wa.chain_ctr, 1u);
        __syncthreads();
        const int sg = uniform(s_seg);
        __syncthreads();
        if (sg >= wa.chain_nseg) break;
        ci.seg = wa.chain_k[sg];
        ci.nseg = wa.chain_nk[sg];
        ci.lc = wa.chain_lc[sg];
        const int i0 = wa.chain_first[sg], i1 = wa.chain_first[sg + 1];
        for (int i = i0; i < i1; ++i) {
            const int code = wa.chain_code[i];
            ci.u = wa.chain_u[i];
            const int par = (i - i0) & 1;
            ci.cur = carry + par * cstride;
            ci.next = carry + (par ^ 1) * cstride;
            if (code & 1) sweep_unit<float, B, 0, 0, true, true, GC, true, NT>(wa, code, blockIdx.x, smem, false, &ci);
            else sweep_unit<float, B, 0, 0, false, true, GC, true, NT>(wa, code, blockIdx.x, smem, false, &ci);
            // the fluxes handed to the next unit are read by any wave of this
            // workgroup in the next item
            __threadfence();
            __syncthreads();
        }
    }
}

template <typename B, int NT>
static void launch_chain(const WinArgs &wa, unsigned nb, size_t lds, hipStream_t st) {
    switch (wa.s.G) {
    case 1: k_sweep_win_chain<B, 1, NT><<<nb, NT, lds, st>>>(wa); break;
    case 2: k_sweep_win_chain<B, 2, NT><<<nb, NT, lds, st>>>(wa); break;
    case 3: k_sweep_win_chain<B, 3, NT><<<nb, NT, lds, st>>>(wa); break;
    case 4: k_sweep_win_chain<B, 4, NT><<<nb, NT, lds, st>>>(wa); break;
    case 5: k_sweep_win_chain<B, 5, NT><<<nb, NT, lds, st>>>(wa); break;
    case 6: k_sweep_win_chain<B, 6, NT><<<nb, NT, lds, st>>>(wa); break;
    case 7: k_sweep_win_chain<B, 7, NT><<<nb, NT, lds, st>>>(wa); break;
    default: k_sweep_win_chain<B, 8, NT><<<nb, NT, lds, st>>>(wa); break;
    }
}

// Store pass of the stored-segment sweep (wa.exp_pass 1 count, 2 step table,
// 3 record): the per-lane walk's geometry only, for any G <= 8.
template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_sweep_win_store(WinArgs wa) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int code = wa.work[blockIdx.x];
    if (code & 1) sweep_unit<float, float, 0, 0, true, true, 0, true, NT, 1>(wa, code, blockIdx.x, smem);
    else sweep_unit<float, float, 0, 0, false, true, 0, true, NT, 1>(wa, code, blockIdx.x, smem);
}

template <typename B, int NT, int EXP = 0, bool PERSIST = false>
static void launch_lane(const WinArgs &wa, unsigned nb, size_t lds, hipStream_t st) {
    switch (wa.s.G) {
    case 1: k_sweep_win_lane<B, 1, NT, EXP, PERSIST><<<nb, NT, lds, st>>>(wa); break;
    case 2: k_sweep_win_lane<B, 2, NT, EXP, PERSIST><<<nb, NT, lds, st>>>(wa); break;
    case 3: k_sweep_win_lane<B, 3, NT, EXP, PERSIST><<<nb, NT, lds, st>>>(wa); break;
    case 4: k_sweep_win_lane<B, 4, NT, EXP, PERSIST><<<nb, NT, lds, st>>>(wa); break;
    case 5: k_sweep_win_lane<B, 5, NT, EXP, PERSIST><<<nb, NT, lds, st>>>(wa); break;
    case 6: k_sweep_win_lane<B, 6, NT, EXP, PERSIST><<<nb, NT, lds, st>>>(wa); break;
    case 7: k_sweep_win_lane<B, 7, NT, EXP, PERSIST><<<nb, NT, lds, st>>>(wa); break;
    default: k_sweep_win_lane<B, 8, NT, EXP, PERSIST><<<nb, NT, lds, st>>>(wa); break;
    }
}

// FP64 arithmetic (precision reference): no register cap
template <typename B, int MODE, bool C1>
__global__ __launch_bounds__(kWinThreads) void k_sweep_win_f64(WinArgs wa) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int code = wa.work[blockIdx.x];
    if (code & 1) sweep_unit<double, B, MODE, 0, true, C1>(wa, code, blockIdx.x, smem);
    else sweep_unit<double, B, MODE, 0, false, C1>(wa, code, blockIdx.x, smem);
}

// Batched form for serving: work unit u0 + b belongs to problem slot
// u_slot[u0 + b] and is (2D track, direction) u_code[u0 + b] of that problem;
// every problem brings its own descriptor (pointers into its own workspace,
// sizes, window length), so the units of all active problems run in one
// launch (one launch per lane layout and workgroup size; one-chunk problems
// take the per-lane walk, shallow ones in 256-thread workgroups).
template <bool C1, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_sweep_win_multi(
    const WinArgs *__restrict__ descs, const int *__restrict__ u_slot, const int *__restrict__ u_code,
    const SlotCtl *__restrict__ ctl, int u0) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int slot = u_slot[u0 + blockIdx.x];
    const int code = u_code[u0 + blockIdx.x];
    if (ctl[slot].done) return;      // stopped: a later step of the batch skips it
    // a descriptor holds the boundary buffers of an even iteration count;
    // problems with an odd count of completed iterations swap them
    const bool flip = (ctl[slot].iters & 1) != 0;
    // descriptors are never written during the launch (restrict): their
    // fields load once instead of after every store to the tallies
    const WinArgs &wa = descs[slot];
    // units of one problem are contiguous in the work list, so neighbouring
    // workgroups mostly run the same specialisation
    if (C1) {
        switch (wa.s.G) {
#define MOC_MULTI_CASE(g)                                                                  \
    case g:                                                                                \
        if (code & 1) sweep_unit<float, float, 0, 0, true, true, g, true, NT>(wa, code, blockIdx.x, smem, flip); \
        else sweep_unit<float, float, 0, 0, false, true, g, true, NT>(wa, code, blockIdx.x, smem, flip);        \
        break;
            MOC_MULTI_CASE(1)
            MOC_MULTI_CASE(2)
            MOC_MULTI_CASE(3)
            MOC_MULTI_CASE(4)
            MOC_MULTI_CASE(5)
            MOC_MULTI_CASE(6)
            MOC_MULTI_CASE(7)
            MOC_MULTI_CASE(8)
#undef MOC_MULTI_CASE
        default: break;
        }
    } else {
        if (code & 1) sweep_unit<float, float, 0, 0, true, false, 0, false, NT>(wa, code, blockIdx.x, smem, flip);
        else sweep_unit<float, float, 0, 0, false, false, 0, false, NT>(wa, code, blockIdx.x, smem, flip);
    }
}

// ------------------------------------------------------------------ F(tau) hook

__global__ void k_eval_attenuation(const float *tau, float *out, long long n, int exp_mode) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = one_minus_exp<float>(tau[i], exp_mode);
}

int eval_attenuation(const float *tau, long long n, int exp_mode, float *out) {
    if (n <= 0) return MOC_OK;
    float *d = nullptr;
    hipError_t e = hipMalloc((void **)&d, (size_t)n * 8);
    if (e != hipSuccess) {
        set_error(hipGetErrorString(e));
        return MOC_ENOMEM;
    }
    e = hipMemcpy(d, tau, (size_t)n * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        k_eval_attenuation<<<(unsigned)((n + 255) / 256), 256>>>(d, d + n, n, exp_mode);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(out, d + n, (size_t)n * 4, hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) {
        set_error(hipGetErrorString(e));
        return MOC_EDEVICE;
    }
    return MOC_OK;
}

// ------------------------------------------------------------------ F(tau) hook without allocation

// Staging of moc_eval_attenuation_noalloc, one copy per device for the life of
// the process: tau in [0, kNoAllocMaxTau), F(tau) in [kNoAllocMaxTau, 2 kNoAllocMaxTau).
// Host code never uses this name as an address: the device address comes from
// hipGetSymbolAddress, once per device, and is kept in g_scratch_dev.
static __device__ __align__(256) float scratch[2 * kNoAllocMaxTau];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_dev[kMaxDevices] = {};
}  // namespace

int eval_attenuation_noalloc(const float *tau, long long n, int exp_mode, float *out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error(hipGetErrorString(e));
        return MOC_EDEVICE;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device index beyond the library's per-device table");
        return MOC_EDEVICE;
    }
    float *buf = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_dev[dev]) {
            void *p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) {
                set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
                return MOC_EDEVICE;
            }
            g_scratch_dev[dev] = static_cast<float *>(p);
        }
        buf = g_scratch_dev[dev];
    }
    if (n <= 0) return MOC_OK;
    // every element read below is written first: nothing has to start at zero
    e = hipMemcpy(buf, tau, (size_t)n * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        k_eval_attenuation<<<(unsigned)((n + 255) / 256), 256>>>(buf, buf + kNoAllocMaxTau, n, exp_mode);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(out, buf + kNoAllocMaxTau, (size_t)n * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        set_error(hipGetErrorString(e));
        return MOC_EDEVICE;
    }
    return MOC_OK;
}

// ------------------------------------------------------------------ trace hook

// One thread per requested stored track (forward): the same piece generation
// as the sweeps, written out instead of swept.
__global__ void k_trace(SweepArgs a, const long long *tracks, long long ntr, int cap, int *fsr,
                        double *len, int *count) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ntr) return;
    const long long trk = tracks[i];
    long long lo = 0, hi = a.n_stacks;
    while (hi - lo > 1) {
        long long mid = (lo + hi) >> 1;
        if (a.trk_off[mid] <= trk) lo = mid;
        else hi = mid;
    }
    const long long s = lo;
    const int P = a.P, K = a.K;
    const long long t = s / P;
    const int n = (int)(s - t * P);
    const int an = (a.t_meta[t] & 0xffff) * P + n;
    const double c = a.cot[an], ic = a.icot[an], secl = a.secl[an];
    const double Lt = a.t_len[t];
    const int f0 = a.t_first[t], f1 = a.t_first[t + 1];
    const double base = line_base(a, s, trk - a.trk_off[s]);
    double ls, le;
    clip_line(base, c, ic, Lt, a.H, ls, le);
    Walker wk;
    walk_init(wk, base, c, ic, a.h, a.inv_h, K, ls, false);
    int m = 0;
    for (int k = seg_search(a.seg_pos, f0, f1, ls); k < f1; ++k) {
        const double s0 = a.seg_pos[k];
        if (s0 >= le) break;
        const double s1 = (k + 1 < f1) ? a.seg_pos[k + 1] : Lt;
        const double e = fmin(s1, le);
        if (!(e > wk.lcur)) continue;
        const long long jb = (long long)a.seg_reg[k] * K;
        walk_segment<false>(wk, e, secl, K, [&](int kz, double l3, bool valid) {
            if (!valid) return;
            if (m < cap) {
                fsr[i * cap + m] = (int)(jb + kz);
                len[i * cap + m] = l3;
            }
            ++m;
        });
    }
    count[i] = m;
}

// ------------------------------------------------------------------ boundary hook

// out[i][g] = buf[slots[i]][g], widened to FP64 (buf holds B values)
template <typename B>
__global__ void k_gather_slots(const B *buf, const long long *slots, long long n, int G, double *out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * G) return;
    const long long k = i / G;
    const int g = (int)(i - k * G);
    out[i] = (double)buf[slots[k] * G + g];
}

// ------------------------------------------------------------------ source / finalize


// qhat = (sum_g' Sigma_s[g'->g] phi_g' + Q_g) / (4 pi Sigma_t,g); clears the tally.
__device__ inline void source_elem(const FsrArgs &a, long long i) {
    if (i >= a.n) return;
    const int G = a.G;
    const long long j = i / G;
    const int g = (int)(i - j * G);
    const int mat = a.reg_mat[j / a.K];
    double sum = a.q[i];
    const double *ph = a.phi + j * G;
    const double *ss = a.sigs + (size_t)mat * G * G + g;
    for (int gp = 0; gp < G; ++gp) sum += ss[(size_t)gp * G] * ph[gp];
    const double qh = sum / (kFourPi * a.sigt[mat * G + g]);
    a.qhat64[i] = qh;
    a.qhat32[i] = (float)qh;
    a.acc[i] = 0.0;
}

// phi = 4 pi qhat + acc / (Sigma_t V) (Eq. 4 estimator); residual and totals.
__device__ inline void finalize_elem(const FsrArgs &a, long long i, int slot_seed) {
    double res = 0.0, bal = 0.0, absb = 0.0, src = 0.0;
    if (i < a.n) {
        const int G = a.G;
        const long long j = i / G;
        const int g = (int)(i - j * G);
        const int mat = a.reg_mat[j / a.K];
        const double st = a.sigt[mat * G + g];
        const double v = a.vol[j];
        const double ac = a.acc[i];
        const double ph = kFourPi * a.qhat64[i] + (v > 0 ? ac / (st * v) : 0.0);
        const double old = a.phi[i];
        const double d = fabs(ph - old);
        res = (ph != 0.0) ? d / fabs(ph) : (d == 0.0 ? 0.0 : 1.0);
        a.phi[i] = ph;
        double out = 0.0;
        const double *ss = a.sigs + ((size_t)mat * G + g) * G;
        for (int gp = 0; gp < G; ++gp) out += ss[gp];
        bal = ac;
        absb = v * (st - out) * ph;
        src = v * a.q[i];
    }
    // block totals (4 waves) -> one set of atomics per block, spread over
    // the slots; the residual is a max over the Q_RES slots (res >= 0, so
    // the bit patterns order like the values)
    res = wave_max(res);
    bal = wave_sum(bal);
    absb = wave_sum(absb);
    src = wave_sum(src);
    __shared__ double red[4][4];
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[wv][0] = res;
        red[wv][1] = bal;
        red[wv][2] = absb;
        red[wv][3] = src;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 1; w < nw; ++w) {
            res = fmax(res, red[w][0]);
            bal += red[w][1];
            absb += red[w][2];
            src += red[w][3];
        }
        const int sl = slot_seed % kSlots;
        atomicMax((unsigned long long *)&a.scal[slot_index(Q_RES, sl)],
                  (unsigned long long)__double_as_longlong(res));
        unsafeAtomicAdd(&a.scal[slot_index(Q_BAL, sl)], bal);
        unsafeAtomicAdd(&a.scal[slot_index(Q_ABS, sl)], absb);
        unsafeAtomicAdd(&a.scal[slot_index(Q_SRC, sl)], src);
    }
}

// Residual of one problem: the max over its Q_RES slots
__device__ inline double residual_of(const double *scal) {
    double r = 0.0;
    for (int sl = 0; sl < kSlots; ++sl) r = fmax(r, scal[slot_index(Q_RES, sl)]);
    return r;
}


// Source update; also clears the scalar block (accumulators of this
// iteration, the finalize ticket) before the sweep adds into it.
__global__ __launch_bounds__(256) void k_source(FsrArgs a, int scal_words) {
    unsigned *sw = (unsigned *)a.scal;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < scal_words; i += gridDim.x * blockDim.x)
        sw[i] = 0u;
    source_elem(a, (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

// The residual of a single solve folded on the device: the max over the
// Q_RES slots into word 0 of the scalar block (never a slot), so the host
// reads 8 bytes.
__global__ void k_fold_residual(double *scal) {
    double r = threadIdx.x < kSlots ? scal[slot_index(Q_RES, threadIdx.x)] : 0.0;
    r = wave_max(r);
    if (threadIdx.x == 0) scal[0] = r;
}

// Finalize; the residual is the max over the Q_RES slots (folded by the
// reader: the host, the single-solve fold or the batched residual gather).
__global__ __launch_bounds__(256) void k_finalize(FsrArgs a) {
    finalize_elem(a, (long long)blockIdx.x * blockDim.x + threadIdx.x, blockIdx.x);
}

// Batched forms: problem slot of a block from the block prefix blk_pre
// (n_slots + 1 entries); the block index inside the problem follows.
__device__ inline int slot_of_block(const int *blk_pre, int n_slots, int b) {
    int lo = 0, hi = n_slots;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (blk_pre[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_source_multi(const FsrArgs *__restrict__ args,
                                                      const int *__restrict__ blk_pre,
                                                      const SlotCtl *__restrict__ ctl, int n_slots) {
    const int sl = slot_of_block(blk_pre, n_slots, blockIdx.x);
    if (ctl[sl].done) return;
    source_elem(args[sl], (long long)(blockIdx.x - blk_pre[sl]) * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(256) void k_finalize_multi(const FsrArgs *__restrict__ args,
                                                        const int *__restrict__ blk_pre,
                                                        const SlotCtl *__restrict__ ctl, int n_slots) {
    const int sl = slot_of_block(blk_pre, n_slots, blockIdx.x);
    if (ctl[sl].done) return;
    const int b = blockIdx.x - blk_pre[sl];
    finalize_elem(args[sl], (long long)b * blockDim.x + threadIdx.x, b);
}

// Clear the scalar block of every running problem (blockIdx.y = slot); a
// stopped one keeps its last iteration's totals.
__global__ void k_clear_scal_multi(const FsrArgs *args, const SlotCtl *ctl, int words) {
    if (ctl[blockIdx.y].done) return;
    unsigned *p = (unsigned *)args[blockIdx.y].scal;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < words; i += gridDim.x * blockDim.x)
        p[i] = 0u;
}

// End of a batched step: the residual of every running problem into one
// compact array, one more completed iteration, and the stopping rule (the
// residual of an iteration after the first below tol, or max_iters reached).
// A stopped problem is skipped by every later step of the batch, so steps
// launched before the host has read this one leave its result as it is.
__global__ void k_gather_residual(const FsrArgs *args, int n_slots, double *out, SlotCtl *ctl) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_slots && !ctl[i].done) {
        const double r = residual_of(args[i].scal);
        const int it = ctl[i].iters + 1;
        out[i] = r;
        ctl[i].iters = it;
        if ((it > 1 && r < ctl[i].tol) || it >= ctl[i].max_iters) ctl[i].done = 1;
    }
}

// ------------------------------------------------------------------ eigenvalue mode

// The fission source chi_g F_j / k in place of the fixed source, with
// F_j = sum_g' nuSigma_f,g' phi_j,g' of the current iterate; F_j is kept for
// the production ratio and the shape residual.
__global__ __launch_bounds__(256) void k_fission_source(FsrArgs a, double *q, const double *nusf,
                                                        const double *chi, double inv_k, double *fold) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int G = a.G;
    const long long j = i / G;
    const int g = (int)(i - j * G);
    const int mat = a.reg_mat[j / a.K];
    const double *ph = a.phi + j * G;
    double F = 0.0;
    for (int gp = 0; gp < G; ++gp) F += nusf[mat * G + gp] * ph[gp];
    q[i] = chi[mat * G + g] * F * inv_k;
    if (g == 0) fold[j] = F;
}

// Fission production of the previous and of the new iterate, sum_j V_j F_j,
// into the Q_POLD / Q_PNEW slots (one atomic per wave).
__global__ __launch_bounds__(256) void k_production(FsrArgs a, const double *nusf, const double *fold) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int G = a.G;
    double pn = 0.0, po = 0.0;
    if (j < a.n / G) {
        const int mat = a.reg_mat[j / a.K];
        double F = 0.0;
        for (int g = 0; g < G; ++g) F += nusf[mat * G + g] * a.phi[j * G + g];
        pn = a.vol[j] * F;
        po = a.vol[j] * fold[j];
    }
    pn = wave_sum(pn);
    po = wave_sum(po);
    if ((threadIdx.x & 63) == 0) {
        const int sl = (int)((blockIdx.x * 4 + (threadIdx.x >> 6)) % kSlots);
        unsafeAtomicAdd(&a.scal[slot_index(Q_PNEW, sl)], pn);
        unsafeAtomicAdd(&a.scal[slot_index(Q_POLD, sl)], po);
    }
}

// Largest change of the normalised fission source over fissile FSRs,
// |F_j(new) r - F_j(old)| / (F_j(new) r) with r = P_old / P_new, into the
// Q_SHAPE slots (a max: the values are >= 0, so their bit patterns order).
__global__ __launch_bounds__(256) void k_shape_residual(FsrArgs a, const double *nusf, const double *fold,
                                                        double ratio) {
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int G = a.G;
    double r = 0.0;
    if (j < a.n / G) {
        const int mat = a.reg_mat[j / a.K];
        double F = 0.0;
        for (int g = 0; g < G; ++g) F += nusf[mat * G + g] * a.phi[j * G + g];
        if (F > 0.0) r = fabs(F * ratio - fold[j]) / (F * ratio);
    }
    r = wave_max(r);
    if ((threadIdx.x & 63) == 0) {
        const int sl = (int)((blockIdx.x * 4 + (threadIdx.x >> 6)) % kSlots);
        atomicMax((unsigned long long *)&a.scal[slot_index(Q_SHAPE, sl)],
                  (unsigned long long)__double_as_longlong(r));
    }
}

__global__ void k_fill_f64(double *p, double v, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_u32(unsigned *p, unsigned v, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// ------------------------------------------------------------------ host side

static thread_local std::string g_err;
void set_error(const std::string &e) { g_err = e; }
const char *last_error() { return g_err.c_str(); }

#define HIPCHK(x)                                                                      \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) {                                                        \
            set_error(std::string(#x) + ": " + hipGetErrorString(e_));                 \
            return MOC_EDEVICE;                                                        \
        }                                                                              \
    } while (0)

int fill_zero(void *p, size_t bytes, hipStream_t st) {
    if (bytes == 0) return MOC_OK;
    size_t n = bytes / 4;
    int blocks = (int)std::min<size_t>((n + 255) / 256, 65536);
    k_fill_u32<<<blocks, 256, 0, st>>>((unsigned *)p, 0u, n);
    HIPCHK(hipGetLastError());
    return MOC_OK;
}

template <typename T>
static T *ws_ptr(char *ws, size_t off) {
    return reinterpret_cast<T *>(ws + off);
}

SweepArgs Solver::sweep_args(int fp64, int exp_mode) const {
    SweepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.cot = ws_ptr<double>(ws, lay.off_cot);
    a.secl = ws_ptr<double>(ws, lay.off_secl);
    a.icot = ws_ptr<double>(ws, lay.off_icot);
    a.inv_dz = 1.0 / info.dz;
    a.wgt = ws_ptr<double>(ws, lay.off_wgt);
    a.t_len = ws_ptr<double>(ws, lay.off_t_len);
    a.t_first = ws_ptr<int>(ws, lay.off_t_first);
    a.t_meta = ws_ptr<int>(ws, lay.off_t_meta);
    a.t_link = ws_ptr<int>(ws, lay.off_t_link);
    a.seg_pos = ws_ptr<double>(ws, lay.off_seg_pos);
    a.seg_reg = ws_ptr<int>(ws, lay.off_seg_reg);
    a.reg_mat = ws_ptr<int>(ws, lay.off_reg_mat);
    a.zeta = ws_ptr<double>(ws, lay.off_zeta);
    a.ilo = ws_ptr<long long>(ws, lay.off_ilo);
    a.cnt = ws_ptr<int>(ws, lay.off_cnt);
    a.trk_off = ws_ptr<long long>(ws, lay.off_trk_off);
    a.chunk_off = ws_ptr<long long>(ws, lay.off_chunk_off);
    a.sigt = fp64 ? (const void *)ws_ptr<double>(ws, lay.off_sigt64)
                  : (const void *)ws_ptr<float>(ws, lay.off_sigt32);
    a.sigt64 = ws_ptr<double>(ws, lay.off_sigt64);
    a.seg_st = ws_ptr<float>(ws, lay.off_seg_st);
    a.qhat = fp64 ? (const void *)ws_ptr<double>(ws, lay.off_qhat64)
                  : (const void *)ws_ptr<float>(ws, lay.off_qhat32);
    a.acc = ws_ptr<double>(ws, lay.off_acc);
    a.scal = ws_ptr<double>(ws, lay.off_scal);
    a.n_items = 2 * info.n_chunks;
    a.n_stacks = info.n_stacks;
    a.H = H;
    a.h = h;
    a.inv_h = 1.0 / h;
    a.dz = info.dz;
    a.G = info.n_groups;
    a.P = P;
    a.K = K;
    a.T = info.tracks_per_wave;
    a.C = group_chunks(a.G);
    a.GL = groups_per_lane(a.G);
    std::memcpy(a.bc, bc, sizeof(a.bc));
    a.exp_mode = exp_mode;
    return a;
}

FsrArgs Solver::fsr_args() const {
    FsrArgs f;
    f.q = ws_ptr<double>(ws, lay.off_q);
    f.sigt = ws_ptr<double>(ws, lay.off_sigt64);
    f.sigs = ws_ptr<double>(ws, lay.off_sigs);
    f.vol = ws_ptr<double>(ws, lay.off_vol);
    f.reg_mat = ws_ptr<int>(ws, lay.off_reg_mat);
    f.phi = ws_ptr<double>(ws, lay.off_phi);
    f.acc = ws_ptr<double>(ws, lay.off_acc);
    f.qhat64 = ws_ptr<double>(ws, lay.off_qhat64);
    f.qhat32 = ws_ptr<float>(ws, lay.off_qhat32);
    f.scal = ws_ptr<double>(ws, lay.off_scal);
    f.n = (long long)info.n_fsr * info.n_groups;
    f.G = info.n_groups;
    f.K = K;
    return f;
}

int Solver::upload(const Plan &p) {
    auto put = [&](size_t off, const void *src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpyAsync(ws + off, src, bytes, hipMemcpyHostToDevice, stream);
    };
    // host staging kept alive until the stream has consumed it
    std::vector<double> secl(p.cot.size()), icot(p.cot.size());
    for (size_t i = 0; i < p.cot.size(); ++i) {
        double c = p.cot[i];
        secl[i] = std::sqrt(1.0 + c * c);   // 3D length per unit 2D length
        icot[i] = 1.0 / c;                  // cot is never 0 (k >= 1 in the polar correction)
    }
    std::vector<int> tfirst(p.n2d + 1), tmeta(p.n2d), tlink(2 * p.n2d);
    for (int64_t t = 0; t <= p.n2d; ++t) tfirst[t] = (int)p.seg_first[t];
    for (int64_t t = 0; t < p.n2d; ++t)
        tmeta[t] = p.az[t] | (p.face0[t] << 16) | (p.face1[t] << 20);
    for (int64_t i = 0; i < 2 * p.n2d; ++i) tlink[i] = (int)p.link[i];
    std::vector<int> cnt(p.n_stacks);
    for (int64_t s = 0; s < p.n_stacks; ++s) cnt[s] = (int)p.cnt[s];
    std::vector<float> sigt32(p.sigt.begin(), p.sigt.end());
    HIPCHK(put(lay.off_cot, p.cot.data(), p.cot.size() * 8));
    HIPCHK(put(lay.off_secl, secl.data(), secl.size() * 8));
    HIPCHK(put(lay.off_icot, icot.data(), icot.size() * 8));
    HIPCHK(put(lay.off_wgt, p.wgt.data(), p.wgt.size() * 8));
    HIPCHK(put(lay.off_t_len, p.L.data(), p.n2d * 8));
    HIPCHK(put(lay.off_t_first, tfirst.data(), tfirst.size() * 4));
    HIPCHK(put(lay.off_t_meta, tmeta.data(), tmeta.size() * 4));
    HIPCHK(put(lay.off_t_link, tlink.data(), tlink.size() * 4));
    HIPCHK(put(lay.off_seg_pos, p.seg_pos.data(), p.seg_pos.size() * 8));
    HIPCHK(put(lay.off_seg_reg, p.seg_reg.data(), p.seg_reg.size() * 4));
    HIPCHK(put(lay.off_reg_mat, p.reg_mat.data(), p.reg_mat.size() * 4));
    HIPCHK(put(lay.off_zeta, p.zeta.data(), p.n_stacks * 8));
    HIPCHK(put(lay.off_ilo, p.ilo.data(), p.n_stacks * 8));
    HIPCHK(put(lay.off_cnt, cnt.data(), cnt.size() * 4));
    HIPCHK(put(lay.off_trk_off, p.trk_off.data(), p.trk_off.size() * 8));
    HIPCHK(put(lay.off_chunk_off, p.chunk_off.data(), p.chunk_off.size() * 8));
    HIPCHK(put(lay.off_ch_first, p.ch_first.data(), p.ch_first.size() * 4));
    HIPCHK(put(lay.off_ch_code, p.ch_code.data(), p.ch_code.size() * 4));
    HIPCHK(put(lay.off_ch_u, p.ch_u.data(), p.ch_u.size() * 8));
    HIPCHK(put(lay.off_ch_k, p.ch_k.data(), p.ch_k.size() * 4));
    HIPCHK(put(lay.off_ch_nk, p.ch_nk.data(), p.ch_nk.size() * 4));
    HIPCHK(put(lay.off_ch_lc, p.ch_lc.data(), p.ch_lc.size() * 8));
    n_chseg = p.n_chseg;
    chain_cap = (int)p.ch_cap;
    HIPCHK(put(lay.off_sigt32, sigt32.data(), sigt32.size() * 4));
    HIPCHK(put(lay.off_sigt64, p.sigt.data(), p.sigt.size() * 8));
    HIPCHK(put(lay.off_sigs, p.sigs.data(), p.sigs.size() * 8));
    {
        // Sigma_t log2(e) of every 2D segment's material, rounded once to FP32
        // (the FP32 sweep copies a window's rows straight into LDS)
        std::vector<float> seg_st(p.seg_reg.size() * (size_t)p.G);
        for (size_t k = 0; k < p.seg_reg.size(); ++k) {
            const int m = p.reg_mat[p.seg_reg[k]];
            for (int g = 0; g < p.G; ++g)
                seg_st[k * p.G + g] = (float)(p.sigt[(size_t)m * p.G + g] * 1.4426950408889634);
        }
        HIPCHK(put(lay.off_seg_st, seg_st.data(), seg_st.size() * 4));
    }
    // windowed sweep: window size from the LDS budget, and the work list of
    // (2D track, direction) units ordered by decreasing work (lines x 2D
    // segments), so the longest units start first
    sw32 = window_fit(p, false);
    sw64 = window_fit(p, true);
    lstride = p.lstride;
    // the per-lane walk was measured faster on shallow and deep stacks alike
    // (lattice8 / 32 / 64); it exists for the one-chunk lane layout
    walk_auto = group_chunks(p.G) == 1 ? 1 : 0;
    walk = walk_auto;
    lane_sw = 0;
    if (walk_auto == 1 && p.P <= kMaxPolar) {
        int max_seg = 1;
        for (int64_t t = 0; t < p.n2d; ++t)
            max_seg = std::max<int>(max_seg, (int)(p.seg_first[t + 1] - p.seg_first[t]));
        int s = 0;
        while (s < max_seg && win_lds_bytes(s + 1, p.K, p.G, 4) <= kWinLdsBudgetSmall) ++s;
        sw256 = s;
        if (s >= kWinSmallMinSw || (s >= 1 && s == max_seg)) lane_sw = s;
        int b = 0;
        while (b < max_seg && win_lds_bytes(b + 1, p.K, p.G, 4) <= kWinLdsBudgetBig) ++b;
        sw1024 = b;
        bpw256 = bundles_per_wave(p, sw256, 256);
        bpw512 = bundles_per_wave(p, sw32, kWinThreads);
        bpw1024 = bundles_per_wave(p, sw1024, kWinThreadsBig);
    }
    choose_lane_window();
    std::vector<std::pair<double, int>> est(p.n2d);
    for (int64_t t = 0; t < p.n2d; ++t) {
        double lines = 0;
        for (int n = 0; n < p.P; ++n) lines += (double)p.cnt[t * p.P + n];
        est[t] = {lines * (double)(p.seg_first[t + 1] - p.seg_first[t]), (int)t};
    }
    std::stable_sort(est.begin(), est.end(), [](const std::pair<double, int> &x,
                                                const std::pair<double, int> &y) {
        return x.first > y.first;
    });
    std::vector<int> work(2 * p.n2d);
    work_cost.resize(2 * p.n2d);
    for (int64_t i = 0; i < p.n2d; ++i) {
        work[2 * i] = 2 * est[i].second;
        work[2 * i + 1] = 2 * est[i].second + 1;
        // in wave passes: a wave carries T lines of all groups
        work_cost[2 * i] = work_cost[2 * i + 1] = (float)(est[i].first / p.T);
    }
    HIPCHK(put(lay.off_work, work.data(), work.size() * 4));
    work_host = work;
    track_work.resize(p.n2d);
    for (int64_t t = 0; t < p.n2d; ++t) track_work[est[t].second] = est[t].first;
    chunk_off.assign(p.chunk_off.begin(), p.chunk_off.end());
    trk_off.assign(p.trk_off.begin(), p.trk_off.end());
    cnt.assign(p.cnt.begin(), p.cnt.end());
    HIPCHK(hipStreamSynchronize(stream));
    return MOC_OK;
}

int Solver::compute_volumes() {
    int rc = fill_zero(ws + lay.off_acc, (size_t)info.n_fsr * 8, stream);
    if (rc) return rc;
    rc = fill_zero(ws + lay.off_scal, 128 * 1024, stream);
    if (rc) return rc;
    SweepArgs a = sweep_args(0, 0);
    a.mode = 1;
    a.psi_in = nullptr;
    a.psi_out = nullptr;
    launch_sweep(a, false);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(ws + lay.off_vol, ws + lay.off_acc, (size_t)info.n_fsr * 8,
                          hipMemcpyDeviceToDevice, stream));
    HIPCHK(hipStreamSynchronize(stream));
    return MOC_OK;
}

template <typename R, typename B, bool C1>
static void launch_win_c(const WinArgs &wa, unsigned nb, size_t lds, hipStream_t st, int mode, int expm) {
    if (std::is_same<R, double>::value) {
        if (mode == 1) k_sweep_win_f64<B, 1, C1><<<nb, kWinThreads, lds, st>>>(wa);
        else k_sweep_win_f64<B, 0, C1><<<nb, kWinThreads, lds, st>>>(wa);
    } else if (mode == 1) {
        k_sweep_win<B, 1, 0, C1><<<nb, kWinThreads, lds, st>>>(wa);
    } else if (expm == 0 && C1 && wa.walk == 1) {
        if (wa.small_wg) launch_lane<B, 256>(wa, nb, lds, st);
        else if (wa.big_wg) launch_lane<B, kWinThreadsBig>(wa, nb, lds, st);
        else launch_lane<B, kWinThreads>(wa, nb, lds, st);
    } else if (expm == 0) {
        // the transport sweep with the group count compiled in (G <= 8)
        switch (C1 ? wa.s.G : 0) {
        case 1: k_sweep_win<B, 0, 0, true, 1><<<nb, kWinThreads, lds, st>>>(wa); break;
        case 2: k_sweep_win<B, 0, 0, true, 2><<<nb, kWinThreads, lds, st>>>(wa); break;
        case 3: k_sweep_win<B, 0, 0, true, 3><<<nb, kWinThreads, lds, st>>>(wa); break;
        case 4: k_sweep_win<B, 0, 0, true, 4><<<nb, kWinThreads, lds, st>>>(wa); break;
        case 5: k_sweep_win<B, 0, 0, true, 5><<<nb, kWinThreads, lds, st>>>(wa); break;
        case 6: k_sweep_win<B, 0, 0, true, 6><<<nb, kWinThreads, lds, st>>>(wa); break;
        case 7: k_sweep_win<B, 0, 0, true, 7><<<nb, kWinThreads, lds, st>>>(wa); break;
        case 8: k_sweep_win<B, 0, 0, true, 8><<<nb, kWinThreads, lds, st>>>(wa); break;
        default: k_sweep_win<B, 0, 0, C1><<<nb, kWinThreads, lds, st>>>(wa); break;
        }
    } else {
        k_sweep_win<B, 0, 1, C1><<<nb, kWinThreads, lds, st>>>(wa);
    }
}

template <typename R, typename B>
static void launch_win(const WinArgs &wa, unsigned nb, size_t lds, hipStream_t st, int mode, int expm) {
    if (wa.s.C == 1) launch_win_c<R, B, true>(wa, nb, lds, st, mode, expm);
    else launch_win_c<R, B, false>(wa, nb, lds, st, mode, expm);
}

// The per-lane FP32 transport sweep of a work list (replay or on-the-fly),
// one workgroup per unit or a persistent grid of at most `grid` workgroups.
template <int EXP>
static void launch_lane_list(WinArgs wa, int n, int grid, size_t lds, bool psi64, hipStream_t st) {
    if (n <= 0) return;
    if (grid > 0 && !psi64) {
        // persistent grid (FP32 boundary storage only)
        wa.persist_units = n;
        const unsigned nb = (unsigned)std::min(n, grid);
        if (wa.small_wg) launch_lane<float, 256, EXP, true>(wa, nb, lds, st);
        else if (wa.big_wg) launch_lane<float, kWinThreadsBig, EXP, true>(wa, nb, lds, st);
        else launch_lane<float, kWinThreads, EXP, true>(wa, nb, lds, st);
        return;
    }
    const unsigned nb = (unsigned)n;
    wa.persist_units = 0;
    if (psi64) {
        if (wa.small_wg) launch_lane<double, 256, EXP>(wa, nb, lds, st);
        else if (wa.big_wg) launch_lane<double, kWinThreadsBig, EXP>(wa, nb, lds, st);
        else launch_lane<double, kWinThreads, EXP>(wa, nb, lds, st);
    } else {
        if (wa.small_wg) launch_lane<float, 256, EXP>(wa, nb, lds, st);
        else if (wa.big_wg) launch_lane<float, kWinThreadsBig, EXP>(wa, nb, lds, st);
        else launch_lane<float, kWinThreads, EXP>(wa, nb, lds, st);
    }
}

// Store pass launch over n units with the lane sweep's workgroup size.
static void launch_store(const WinArgs &wa, int n, size_t lds, hipStream_t st) {
    if (wa.small_wg) k_sweep_win_store<256><<<n, 256, lds, st>>>(wa);
    else if (wa.big_wg) k_sweep_win_store<kWinThreadsBig><<<n, kWinThreadsBig, lds, st>>>(wa);
    else k_sweep_win_store<kWinThreads><<<n, kWinThreads, lds, st>>>(wa);
}

bool Solver::lane_path(const SweepArgs &a, bool fp64) const {
    return !fp64 && a.mode == 0 && a.exp_mode == 0 && walk == 1 && group_chunks(info.n_groups) == 1 &&
           lane_win >= 1;
}

// Dynamic bundle assignment pays where a window holds many bundles of
// unequal length per wave (measured: lattice64, about 16 bundles per wave,
// 10% faster; lattice32 in 256- and 512-thread windows, 5 to 10 per wave,
// 1-2% faster); with two or three per wave the static order was as fast or
// faster (lattice8, lattice32 in 1024-thread windows).
constexpr double kDynBundlesPerWave = 4.0;
bool Solver::dyn_bundles() const {
    if (bundles >= 0) return bundles == 1;
    const double bpw = lane_nt == 256 ? bpw256 : lane_nt == kWinThreadsBig ? bpw1024 : bpw512;
    return bpw >= kDynBundlesPerWave;
}

// Mean number of 64-line bundles per wave in a window of Sw 2D segments swept
// by nt threads, each window weighted by its line count (a window's time
// grows with its lines), over up to 256 2D tracks spread through the plan.
// A line z = base + cot l of a stack crosses the window [wa, wb] when its
// base lies in an open interval of the two ends; the count of evenly spaced
// bases in it is rounded, as suits an estimate.
double bundles_per_wave(const Plan &p, int Sw, int nt) {
    if (Sw < 1 || p.n2d < 1) return 0.0;
    const int64_t step = std::max<int64_t>(1, p.n2d / 256);
    double num = 0.0, den = 0.0;
    for (int64_t t = 0; t < p.n2d; t += step) {
        const int64_t f0 = p.seg_first[t], f1 = p.seg_first[t + 1];
        for (int64_t k0 = f0; k0 < f1; k0 += Sw) {
            const int64_t k1 = std::min<int64_t>(k0 + Sw, f1);
            const double wa = p.seg_pos[k0], wb = k1 < f1 ? p.seg_pos[k1] : p.L[t];
            double lines = 0.0;
            for (int n = 0; n < p.P; ++n) {
                const int64_t s = t * p.P + n;
                const double c = p.cot[p.az[t] * p.P + n];
                const double lo = c > 0 ? -wb * c : -wa * c, hi = c > 0 ? p.H - wa * c : p.H - wb * c;
                const double z0 = p.zeta[s] + (double)p.ilo[s] * p.dz;
                const double i0 = std::max(0.0, std::ceil((lo - z0) / p.dz));
                const double i1 = std::min((double)p.cnt[s] - 1.0, std::floor((hi - z0) / p.dz));
                if (i1 >= i0) lines += i1 - i0 + 1.0;
            }
            num += lines * lines;
            den += lines;
        }
    }
    return den > 0.0 ? num / den / 64.0 / (nt / 64) : 0.0;
}

WinArgs Solver::lane_args(const SweepArgs &a) const {
    WinArgs wa;
    std::memset(&wa, 0, sizeof(wa));
    wa.s = a;
    wa.small_wg = lane_nt == 256 ? 1 : 0;
    wa.big_wg = lane_nt == kWinThreadsBig ? 1 : 0;
    wa.dyn_bundles = dyn_bundles() ? 1 : 0;
    wa.Sw = lane_win;
    wa.lstride = lstride;
    wa.walk = walk;
    return wa;
}

// Workgroup size and window of the single solver's per-lane sweep: 256
// threads on shallow stacks (the 40 KB window holds kWinSmallMinSw segments,
// or a whole track), 1024 threads on deep ones (the 512-thread window holds
// fewer than kWinBigBelow segments and the 156 KB one at least twice as
// many), else 512; or the size the caller chose (moc_solver_set_window).
void Solver::choose_lane_window() {
    lane_nt = kWinThreads;
    lane_win = sw32;
    if (group_chunks(info.n_groups) != 1) return;
    if (window_nt == 256 && sw256 >= 1) {
        lane_nt = 256;
        lane_win = sw256;
    } else if (window_nt == kWinThreadsBig && sw1024 >= 1) {
        lane_nt = kWinThreadsBig;
        lane_win = sw1024;
    } else if (window_nt == 0) {
        if (lane_sw >= 1) {
            lane_nt = 256;
            lane_win = lane_sw;
        } else if (sw32 >= 1 && sw32 < kWinBigBelow && sw1024 >= 2 * sw32) {
            lane_nt = kWinThreadsBig;
            lane_win = sw1024;
        }
    }
}

int Solver::set_chain(int on) {
    if (chain_only && !on) return MOC_EINVAL;
    if (on) {
        // vacuum top and bottom (every line ends on a z face), and the
        // per-lane FP32 sweep (one group chunk)
        if (n_chseg == 0 || group_chunks(info.n_groups) != 1 || lane_win < 1 || (P % 2) != 0)
            return MOC_EINVAL;
    }
    chain = on;
    drop_step_graphs();
    return MOC_OK;
}

int Solver::set_window(int threads) {
    if (threads == 256 && sw256 < 1) return MOC_EINVAL;
    if (threads == kWinThreadsBig && sw1024 < 1) return MOC_EINVAL;
    window_nt = threads;
    choose_lane_window();
    drop_store();
    drop_step_graphs();
    return MOC_OK;
}

// Workgroups of the lane sweep resident on the device at once: the LDS of a
// workgroup and 16 waves per CU (amdgpu_waves_per_eu(4) on 4 SIMDs).
int Solver::resident_workgroups() const {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const size_t lds = win_lds_bytes(std::max(lane_win, 1), K, info.n_groups, 4);
    const int by_lds = (int)std::max<size_t>(1, (160 * 1024) / std::max<size_t>(lds, 1));
    const int by_waves = std::max(1, 16 / (lane_nt / 64));
    return cus * std::min(by_lds, by_waves);
}

void Solver::launch_sweep(SweepArgs a, bool fp64, const int *units, int n_units,
                          const int *filt_n, const long long *filt_i0) {
    int sw = window_size(fp64);
    // the per-lane walk runs in its own workgroup size and window
    const bool lane = !fp64 && a.mode == 0 && a.exp_mode == 0 && walk == 1 && lane_win >= 1;
    if (lane) sw = lane_win;
    if (!units && chain && lane_path(a, fp64)) {
        // chain-line sweep: per-workgroup carry buffers, no boundary buffer
        WinArgs wa = lane_args(a);
        wa.s.psi_in = nullptr;
        wa.s.psi_out = nullptr;
        wa.chain_nseg = (int)n_chseg;
        wa.chain_cap = chain_cap;
        wa.chain_carry = ws + lay.off_ch_carry;
        wa.chain_first = ws_ptr<int>(ws, lay.off_ch_first);
        wa.chain_code = ws_ptr<int>(ws, lay.off_ch_code);
        wa.chain_u = ws_ptr<double>(ws, lay.off_ch_u);
        wa.chain_k = ws_ptr<int>(ws, lay.off_ch_k);
        wa.chain_nk = ws_ptr<int>(ws, lay.off_ch_nk);
        wa.chain_lc = ws_ptr<double>(ws, lay.off_ch_lc);
        wa.chain_ctr = ws_ptr<unsigned>(ws, lay.off_ch_ctr);
        const unsigned nb = (unsigned)std::min<long long>(
            std::min<long long>(n_chseg, kChainSlots), (long long)resident_workgroups());
        if (nb == 0) return;
        // the segment counter starts from zero (a kernel, also inside a captured graph)
        k_fill_u32<<<1, 64, 0, stream>>>(wa.chain_ctr, 0u, 1);
        const size_t lds = win_lds_bytes(wa.Sw, K, info.n_groups, 4);
        if (lay.psi64) {
            if (wa.small_wg) launch_chain<double, 256>(wa, nb, lds, stream);
            else if (wa.big_wg) launch_chain<double, kWinThreadsBig>(wa, nb, lds, stream);
            else launch_chain<double, kWinThreads>(wa, nb, lds, stream);
        } else {
            if (wa.small_wg) launch_chain<float, 256>(wa, nb, lds, stream);
            else if (wa.big_wg) launch_chain<float, kWinThreadsBig>(wa, nb, lds, stream);
            else launch_chain<float, kWinThreads>(wa, nb, lds, stream);
        }
        return;
    }
    if (!units && lane_path(a, fp64) && (exp_units > 0 || persistent)) {
        // stored-segment sweep: the stored units replayed, then the rest on
        // the fly (two launches in order on the stream); or a persistent grid
        WinArgs wa = lane_args(a);
        const size_t lds = win_lds_bytes(wa.Sw, K, info.n_groups, 4);
        const int grid = persistent ? resident_workgroups() : 0;
        if (exp_units > 0) {
            WinArgs wr = wa;
            wr.work = d_exp_work;
            wr.exp_tbase = d_exp_tbase;
            wr.exp_table = d_exp_table;
            wr.exp_data = d_exp_data;
            launch_lane_list<2>(wr, exp_units, grid, lds, lay.psi64, stream);
            wa.work = d_otf_work;
            launch_lane_list<0>(wa, otf_units, grid, lds, lay.psi64, stream);
        } else {
            wa.work = ws_ptr<int>(ws, lay.off_work);
            launch_lane_list<0>(wa, (int)(2 * info.n_2d_tracks), grid, lds, lay.psi64, stream);
        }
        return;
    }
    if (sw >= 1) {
        WinArgs wa;
        std::memset(&wa, 0, sizeof(wa));
        wa.s = a;
        wa.small_wg = (lane && lane_nt == 256) ? 1 : 0;
        wa.big_wg = (lane && lane_nt == kWinThreadsBig) ? 1 : 0;
        wa.dyn_bundles = (lane && dyn_bundles()) ? 1 : 0;
        wa.work = units ? units : ws_ptr<int>(ws, lay.off_work);
        wa.filt_n = filt_n;
        wa.filt_i0 = filt_i0;
        wa.Sw = sw;
        wa.lstride = lstride;
        wa.walk = walk;
        const unsigned nb = units ? (unsigned)n_units : (unsigned)(2 * info.n_2d_tracks);
        if (nb == 0) return;
        const size_t lds = win_lds_bytes(sw, K, info.n_groups, fp64 ? 8 : 4);
        if (lay.psi64) {
            if (fp64) launch_win<double, double>(wa, nb, lds, stream, a.mode, a.exp_mode);
            else launch_win<float, double>(wa, nb, lds, stream, a.mode, a.exp_mode);
        } else {
            if (fp64) launch_win<double, float>(wa, nb, lds, stream, a.mode, a.exp_mode);
            else launch_win<float, float>(wa, nb, lds, stream, a.mode, a.exp_mode);
        }
        return;
    }
    const long long n = a.n_items;
    if (n <= 0) return;
    const int waves_per_block = 4;
    const long long blocks = (n + waves_per_block - 1) / waves_per_block;
    const dim3 grid((unsigned)blocks);
    if (lay.psi64) {
        if (fp64) k_sweep<double, double><<<grid, 256, 0, stream>>>(a);
        else k_sweep<float, double><<<grid, 256, 0, stream>>>(a);
    } else {
        if (fp64) k_sweep<double, float><<<grid, 256, 0, stream>>>(a);
        else k_sweep<float, float><<<grid, 256, 0, stream>>>(a);
    }
}

// Work units (2 per 2D track) in the order of the schedule.
static std::vector<int> ordered_units(const std::vector<double> &track_work, int order, int group) {
    const int64_t n2d = (int64_t)track_work.size();
    std::vector<int> codes(2 * n2d);
    for (int64_t i = 0; i < 2 * n2d; ++i) codes[i] = (int)i;
    if (order == 1) return codes;     // natural: 2D track order (Eq. 13), both directions
    std::stable_sort(codes.begin(), codes.end(), [&](int x, int y) {
        return track_work[x >> 1] > track_work[y >> 1];
    });
    if (order == 2 && group > 0) {
        // groups of `group` units by decreasing work, every other group reversed
        for (int64_t g0 = group, k = 1; g0 < 2 * n2d; g0 += group, ++k)
            if (k & 1) std::reverse(codes.begin() + g0, codes.begin() + std::min<int64_t>(g0 + group, 2 * n2d));
    }
    return codes;
}

int Solver::upload_work_list() {
    const std::vector<int> codes = ordered_units(track_work, order, resident_workgroups());
    HIPCHK(hipMemcpyAsync(ws + lay.off_work, codes.data(), codes.size() * 4, hipMemcpyHostToDevice, stream));
    HIPCHK(hipStreamSynchronize(stream));
    return MOC_OK;
}

int Solver::set_schedule(int ord, int pers) {
    order = ord;
    persistent = pers;
    drop_store();          // the store's lists follow the order: store again
    drop_step_graphs();
    return upload_work_list();
}

// Stored-segment sweep (paper section 4.2).  A count pass walks every unit's
// geometry once and gives its wave steps and bundle windows; the units with
// the largest footprint are taken, in decreasing order, while they fit the
// caller's buffer; a table pass writes the step count of each of their bundle
// windows, whose exclusive prefix gives each window's place in the store; a
// record pass writes every lane's pieces there.  Buffer layout (256-byte
// aligned parts): stored unit codes, remaining unit codes, table base per
// stored unit, step table (+1 terminal entry), pieces [wave step][64 lanes].
int Solver::store_segments(char *buf, size_t bytes, moc_store_info *out) {
    drop_store();
    drop_step_graphs();
    moc_store_info inf{};
    const int n_units = (int)(2 * info.n_2d_tracks);
    inf.units_total = n_units;
    if (out) *out = inf;
    if (!buf || bytes == 0) return MOC_OK;
    SweepArgs a = sweep_args(0, 0);
    if (!lane_path(a, false)) {
        set_error("the stored-segment sweep records the per-lane FP32 walk (G <= 8, windowed sweep)");
        return MOC_EINVAL;
    }
    WinArgs wa = lane_args(a);
    if ((size_t)wa.Sw * K * info.n_groups >= 65536 || wa.Sw >= 65536) {
        set_error("window too large for the 16-bit piece indices of the store");
        return MOC_EINVAL;
    }
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t lds = win_lds_bytes(wa.Sw, K, info.n_groups, 4);
    // ---- count pass over every unit (in the schedule's order)
    const size_t cnt_bytes = al((size_t)n_units * 16);
    if (bytes < cnt_bytes + al((size_t)n_units * 4)) return MOC_OK;   // too small to count
    std::vector<int> codes = ordered_units(track_work, order, resident_workgroups());
    int *d_codes = reinterpret_cast<int *>(buf + cnt_bytes);
    unsigned long long *d_cnt = reinterpret_cast<unsigned long long *>(buf);
    HIPCHK(hipMemcpyAsync(d_codes, codes.data(), (size_t)n_units * 4, hipMemcpyHostToDevice, stream));
    int rc = fill_zero(d_cnt, (size_t)n_units * 16, stream);
    if (rc) return rc;
    wa.work = d_codes;
    wa.exp_pass = 1;
    wa.exp_count = d_cnt;
    launch_store(wa, n_units, lds, stream);
    HIPCHK(hipGetLastError());
    std::vector<unsigned long long> cnt((size_t)n_units * 2);
    HIPCHK(hipMemcpyAsync(cnt.data(), d_cnt, cnt.size() * 8, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    // ---- choose: decreasing footprint while the total fits
    unsigned long long steps_all = 0;
    std::vector<int> pos(n_units);
    for (int i = 0; i < n_units; ++i) {
        pos[i] = i;
        steps_all += cnt[2 * (size_t)i];
    }
    auto foot = [&](int i) { return cnt[2 * (size_t)i] * 64ull * sizeof(Piece) + cnt[2 * (size_t)i + 1] * 4ull; };
    std::stable_sort(pos.begin(), pos.end(), [&](int x, int y) { return foot(x) > foot(y); });
    const size_t fixed = al((size_t)n_units * 4) * 2 + al((size_t)n_units * 4) + 4096;
    {
        unsigned long long all = 0;
        for (int i = 0; i < n_units; ++i) all += foot(i);
        inf.bytes_all = fixed + (size_t)all + 256 * 3;
    }
    size_t used = 0;
    unsigned long long bw_tot = 0, steps_tot = 0;
    std::vector<char> take(n_units, 0);
    int ns = 0;
    for (int i : pos) {
        const size_t need = (size_t)foot(i);
        if (fixed + used + need + 256 * 3 > bytes) break;     // the paper stops at the budget
        if (steps_tot + cnt[2 * (size_t)i] >= (1ull << 32)) break;
        used += need;
        bw_tot += cnt[2 * (size_t)i + 1];
        steps_tot += cnt[2 * (size_t)i];
        take[i] = 1;
        ++ns;
    }
    inf.wave_steps_total = steps_all;
    if (ns == 0) {
        if (out) *out = inf;
        return MOC_OK;
    }
    // stored and remaining units, each in the schedule's order
    std::vector<int> s_codes, o_codes;
    std::vector<unsigned> tbase;
    unsigned long long run = 0;
    for (int i = 0; i < n_units; ++i) {
        if (take[i]) {
            s_codes.push_back(codes[i]);
            tbase.push_back((unsigned)run);
            run += cnt[2 * (size_t)i + 1];
        } else {
            o_codes.push_back(codes[i]);
        }
    }
    size_t off = 0;
    const size_t o_scodes = off; off += al(s_codes.size() * 4);
    const size_t o_ocodes = off; off += al(std::max<size_t>(o_codes.size(), 1) * 4);
    const size_t o_tbase = off; off += al(tbase.size() * 4);
    const size_t o_table = off; off += al((bw_tot + 1) * 4);
    const size_t o_data = off; off += (size_t)steps_tot * 64 * sizeof(Piece);
    if (off > bytes) {
        set_error("store layout exceeds the buffer");
        return MOC_ENOMEM;
    }
    HIPCHK(hipMemcpyAsync(buf + o_scodes, s_codes.data(), s_codes.size() * 4, hipMemcpyHostToDevice, stream));
    if (!o_codes.empty())
        HIPCHK(hipMemcpyAsync(buf + o_ocodes, o_codes.data(), o_codes.size() * 4, hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(buf + o_tbase, tbase.data(), tbase.size() * 4, hipMemcpyHostToDevice, stream));
    unsigned *d_table = reinterpret_cast<unsigned *>(buf + o_table);
    // ---- table pass: step count of every bundle window of the stored units
    wa.work = reinterpret_cast<int *>(buf + o_scodes);
    wa.exp_tbase = reinterpret_cast<unsigned *>(buf + o_tbase);
    wa.exp_table = d_table;
    wa.exp_count = nullptr;
    wa.exp_pass = 2;
    launch_store(wa, ns, lds, stream);
    HIPCHK(hipGetLastError());
    std::vector<unsigned> table(bw_tot + 1);
    HIPCHK(hipMemcpyAsync(table.data(), d_table, bw_tot * 4, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    unsigned long long acc = 0;
    for (unsigned long long i = 0; i < bw_tot; ++i) {
        const unsigned long long st = table[i];
        table[i] = (unsigned)acc;
        acc += st;
    }
    table[bw_tot] = (unsigned)acc;
    if (acc != steps_tot) {
        set_error("stored-segment step table disagrees with the count pass");
        return MOC_EDEVICE;
    }
    HIPCHK(hipMemcpyAsync(d_table, table.data(), table.size() * 4, hipMemcpyHostToDevice, stream));
    // ---- record pass
    wa.exp_pass = 3;
    wa.exp_data = reinterpret_cast<Piece *>(buf + o_data);
    launch_store(wa, ns, lds, stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream));
    exp_units = ns;
    otf_units = (int)o_codes.size();
    d_exp_work = reinterpret_cast<int *>(buf + o_scodes);
    d_otf_work = reinterpret_cast<int *>(buf + o_ocodes);
    d_exp_tbase = reinterpret_cast<unsigned *>(buf + o_tbase);
    d_exp_table = d_table;
    d_exp_data = wa.exp_data;
    inf.units_stored = ns;
    inf.wave_steps_stored = steps_tot;
    inf.bytes_used = off;
    if (out) *out = inf;
    return MOC_OK;
}

int window_fit(const Plan &p, bool fp64) {
    if (p.P > kMaxPolar) return 0;
    int max_seg = 1;
    for (int64_t t = 0; t < p.n2d; ++t)
        max_seg = std::max<int>(max_seg, (int)(p.seg_first[t + 1] - p.seg_first[t]));
    const int rb = fp64 ? 8 : 4;
    int sw = 0;
    while (sw < max_seg && win_lds_bytes(sw + 1, p.K, p.G, rb) <= kWinLdsBudget) ++sw;
    if (sw < kWinDeepBelow)
        while (sw < max_seg && win_lds_bytes(sw + 1, p.K, p.G, rb) <= kWinLdsBudgetDeep) ++sw;
    return sw;
}

int Solver::init(const Plan &p, char *workspace, size_t ws_bytes, hipStream_t st) {
    info = p.info();
    lay = make_layout(p, ws_bytes >= info.workspace_bytes_fp64);
    chain_only = false;
    if (ws_bytes < lay.total) {
        // chain-only: everything but the boundary buffers, which come last
        if (info.workspace_bytes_chain > 0 && ws_bytes >= info.workspace_bytes_chain) {
            chain_only = true;
        } else {
            set_error("workspace smaller than moc_plan_info.workspace_bytes (and than "
                      "workspace_bytes_chain)");
            return MOC_ENOMEM;
        }
    }
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) {
        set_error("workspace must be 256-byte aligned");
        return MOC_EINVAL;
    }
    ws = workspace;
    stream = st;
    P = p.P;
    K = p.K;
    n_materials = p.M;
    H = p.H;
    h = p.h;
    std::memcpy(bc, p.bc, sizeof(bc));
    int rc = upload(p);
    if (!rc) rc = fill_zero(ws + lay.off_q, (size_t)p.n_fsr * p.G * 8, stream);
    if (!rc) rc = compute_volumes();
    if (!rc) rc = reset();
    if (!rc && chain_only) {
        chain_only = false;
        rc = set_chain(1);
        chain_only = true;
        if (rc) set_error("a chain-only workspace needs the per-lane FP32 sweep (at most 8 groups)");
    }
    return rc;
}

WinArgs Solver::win_args_batched() const {
    WinArgs wa;
    std::memset(&wa, 0, sizeof(wa));
    wa.s = sweep_args(0, 0);
    // buffers of an iteration that follows an even number of completed ones
    // (the batched sweep swaps them after an odd number)
    wa.s.psi_in = ws + lay.off_psi0;
    wa.s.psi_out = ws + lay.off_psi1;
    wa.work = ws_ptr<int>(ws, lay.off_work);
    wa.Sw = sw32;
    wa.lstride = lstride;
    return wa;
}

size_t Solver::win_lds() const { return win_lds_bytes(sw32, K, info.n_groups, 4); }
size_t Solver::lane_lds() const { return win_lds_bytes(lane_sw, K, info.n_groups, 4); }

int launch_batch_step(const BatchStep &b, hipStream_t st) {
    if (b.n_slots <= 0) return MOC_OK;
    k_clear_scal_multi<<<dim3(8, b.n_slots), 256, 0, st>>>(b.fsr_table, b.ctl, 128 * 1024 / 4);
    k_source_multi<<<b.fsr_blocks, 256, 0, st>>>(b.fsr_table, b.blk_pre, b.ctl, b.n_slots);
    if (b.n_units_small > 0)
        k_sweep_win_multi<true, 256><<<b.n_units_small, 256, b.lds_small, st>>>(b.win_table, b.u_slot,
                                                                               b.u_code, b.ctl, 0);
    if (b.n_units_c1 > b.n_units_small)
        k_sweep_win_multi<true, kWinThreads><<<b.n_units_c1 - b.n_units_small, kWinThreads, b.lds, st>>>(
            b.win_table, b.u_slot, b.u_code, b.ctl, b.n_units_small);
    if (b.n_units > b.n_units_c1)
        k_sweep_win_multi<false, kWinThreads><<<b.n_units - b.n_units_c1, kWinThreads, b.lds, st>>>(
            b.win_table, b.u_slot, b.u_code, b.ctl, b.n_units_c1);
    k_finalize_multi<<<b.fsr_blocks, 256, 0, st>>>(b.fsr_table, b.blk_pre, b.ctl, b.n_slots);
    k_gather_residual<<<(b.n_slots + 255) / 256, 256, 0, st>>>(b.fsr_table, b.n_slots, b.res_dev, b.ctl);
    HIPCHK(hipGetLastError());
    return MOC_OK;
}

int Solver::reset() {
    int rc = fill_zero(ws + lay.off_phi, (size_t)info.n_fsr * info.n_groups * 8, stream);
    if (!rc && !chain_only) rc = fill_zero(ws + lay.off_psi0, lay.psi_bytes, stream);
    iter = 0;
    sweep_ms.clear();
    return rc;
}

int Solver::iterate(int nit, const moc_solve_opts &o, bool time_sweep) {
    // the chain-line sweep runs only in the per-lane FP32 transport sweep
    if (chain && !lane_path(sweep_args(o.sweep_fp64, o.exp_mode), o.sweep_fp64 != 0)) {
        set_error("chain mode runs the per-lane FP32 sweep only (no FP64 sweep, no naive exponential)");
        return MOC_EINVAL;
    }
    const FsrArgs f = fsr_args();
    const long long nfg = f.n;
    const unsigned fblocks = (unsigned)((nfg + 255) / 256);
    if (time_sweep) {
        while (events.size() < (size_t)2 * nit) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            events.push_back(e);
        }
    }
    for (int it = 0; it < nit; ++it) {
        ++iter;
        k_source<<<fblocks, 256, 0, stream>>>(f, (int)(kScalBytes / 4));
        SweepArgs a = sweep_args(o.sweep_fp64, o.exp_mode);
        const bool odd = (iter % 2) == 1;
        a.psi_in = ws + (odd ? lay.off_psi0 : lay.off_psi1);
        a.psi_out = ws + (odd ? lay.off_psi1 : lay.off_psi0);
        if (time_sweep) HIPCHK(hipEventRecord(events[2 * it], stream));
        launch_sweep(a, o.sweep_fp64 != 0);
        if (time_sweep) HIPCHK(hipEventRecord(events[2 * it + 1], stream));
        k_finalize<<<fblocks, 256, 0, stream>>>(f);
        HIPCHK(hipGetLastError());
    }
    if (time_sweep) {
        HIPCHK(hipEventSynchronize(events[2 * nit - 1]));
        for (int it = 0; it < nit; ++it) {
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, events[2 * it], events[2 * it + 1]));
            sweep_ms.push_back(ms);
        }
    }
    return MOC_OK;
}

void Solver::drop_step_graphs() {
    for (int b = 0; b < 2; ++b)
        if (step_exec[b]) {
            (void)hipGraphExecDestroy(step_exec[b]);
            step_exec[b] = nullptr;
        }
    step_key = -1;
}

int Solver::solve_step(const moc_solve_opts &o, double *res) {
    // the chain-line sweep runs only in the per-lane FP32 transport sweep
    if (chain && !lane_path(sweep_args(o.sweep_fp64, o.exp_mode), o.sweep_fp64 != 0)) {
        set_error("chain mode runs the per-lane FP32 sweep only (no FP64 sweep, no naive exponential)");
        return MOC_EINVAL;
    }
    const int key = (o.sweep_fp64 ? 1 : 0) | (o.exp_mode ? 2 : 0) | (walk << 2);
    if (!h_res) HIPCHK(hipHostMalloc((void **)&h_res, 64, hipHostMallocDefault));
    for (int b = 0; b < 2; ++b)
        if (!step_ev[b]) HIPCHK(hipEventCreate(&step_ev[b]));
    const FsrArgs f = fsr_args();
    const unsigned fblocks = (unsigned)((f.n + 255) / 256);
    // the launches of one iteration whose sweep reads psi0 (odd) or psi1 (even);
    // launched one by one, the sweep alone sits between the timing events
    auto issue = [&](bool odd, bool timed) -> int {
        k_source<<<fblocks, 256, 0, stream>>>(f, (int)(kScalBytes / 4));
        SweepArgs a = sweep_args(o.sweep_fp64, o.exp_mode);
        a.psi_in = ws + (odd ? lay.off_psi0 : lay.off_psi1);
        a.psi_out = ws + (odd ? lay.off_psi1 : lay.off_psi0);
        if (timed) HIPCHK(hipEventRecord(step_ev[0], stream));
        launch_sweep(a, o.sweep_fp64 != 0);
        if (timed) HIPCHK(hipEventRecord(step_ev[1], stream));
        k_finalize<<<fblocks, 256, 0, stream>>>(f);
        k_fold_residual<<<1, 64, 0, stream>>>(f.scal);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(h_res, f.scal, 8, hipMemcpyDeviceToHost, stream));
        return MOC_OK;
    };
    ++iter;
    const bool odd = (iter % 2) == 1;
    if (stream && !step_graphs_failed) {
        if (key != step_key) {
            drop_step_graphs();
            for (int b = 0; b < 2 && !step_graphs_failed; ++b) {
                hipGraph_t g = nullptr;
                if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                    step_graphs_failed = true;
                    break;
                }
                const int rc = issue(b == 1, false);
                const hipError_t e = hipStreamEndCapture(stream, &g);
                if (rc || e != hipSuccess || !g ||
                    hipGraphInstantiate(&step_exec[b], g, nullptr, nullptr, 0) != hipSuccess)
                    step_graphs_failed = true;
                if (g) (void)hipGraphDestroy(g);
            }
            (void)hipGetLastError();
            if (step_graphs_failed) drop_step_graphs();
            else step_key = key;
        }
    }
    if (step_exec[odd ? 1 : 0]) {
        // a captured iteration is timed as a whole (timing events are not
        // recorded inside the graph)
        HIPCHK(hipEventRecord(step_ev[0], stream));
        HIPCHK(hipGraphLaunch(step_exec[odd ? 1 : 0], stream));
        HIPCHK(hipEventRecord(step_ev[1], stream));
    } else {
        const int rc = issue(odd, true);
        if (rc) return rc;
    }
    HIPCHK(hipStreamSynchronize(stream));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, step_ev[0], step_ev[1]));
    sweep_ms.push_back(ms);
    *res = (iter <= 1) ? 1.0 : *h_res;
    return MOC_OK;
}

Solver::~Solver() {
    drop_step_graphs();
    for (int b = 0; b < 2; ++b)
        if (step_ev[b]) (void)hipEventDestroy(step_ev[b]);
    if (h_res) (void)hipHostFree(h_res);
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
}

int Solver::read_stats(moc_stats *st) {
    std::vector<double> sc(128 * 1024 / 8);
    HIPCHK(hipMemcpyAsync(sc.data(), ws + lay.off_scal, 128 * 1024, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    auto sum = [&](int q) {
        double v = 0;
        for (int i = 0; i < kSlots; ++i) v += sc[slot_index(q, i)];
        return v;
    };
    auto sumu = [&](int q) {
        unsigned long long v = 0;
        for (int i = 0; i < kSlots; ++i) {
            unsigned long long u;
            std::memcpy(&u, &sc[slot_index(q, i)], 8);
            v += u;
        }
        return v;
    };
    std::memset(st, 0, sizeof(*st));
    st->iters = iter;
    double rmax = 0.0;
    for (int i = 0; i < kSlots; ++i) rmax = std::max(rmax, sc[slot_index(Q_RES, i)]);
    st->residual = (iter <= 1) ? 1.0 : rmax;
    st->balance_lhs = sum(Q_BAL);
    st->balance_rhs = sum(Q_SIN) - sum(Q_SOUT);
    st->absorption = sum(Q_ABS);
    st->leakage = sum(Q_LEAK);
    st->source = sum(Q_SRC);
    st->seg_group_updates = sumu(Q_NSEG);
    st->link_errors = sumu(Q_LINKERR);
    if (!sweep_ms.empty()) {
        std::vector<float> v = sweep_ms;
        std::nth_element(v.begin(), v.begin() + v.size() / 2, v.end());
        st->sweep_ms_median = v[v.size() / 2];
    }
    return MOC_OK;
}

// Eigenvalue mode: power iteration on k-eff.  From phi = 1, psi = 0, k = 1,
// every iteration puts the fission source of the current iterate in place of
// the fixed source, runs one source iteration (source update, sweep,
// finalize), updates k by the ratio of fission production and takes as
// residual the larger of the relative change of k and the largest change of
// the normalised fission source (1 at the first iteration).
int Solver::solve_eigen(const double *nusf, const double *chi, const moc_solve_opts &o, double *k_out,
                        double *res_out, int *iters_out) {
    // the chain-line sweep runs only in the per-lane FP32 transport sweep
    if (chain && !lane_path(sweep_args(o.sweep_fp64, o.exp_mode), o.sweep_fp64 != 0)) {
        set_error("chain mode runs the per-lane FP32 sweep only (no FP64 sweep, no naive exponential)");
        return MOC_EINVAL;
    }
    const int G = info.n_groups;
    const size_t mg = (size_t)n_materials * G;
    double *d_nusf = ws_ptr<double>(ws, lay.off_nusf), *d_chi = ws_ptr<double>(ws, lay.off_chi);
    double *d_fold = ws_ptr<double>(ws, lay.off_fold), *d_q = ws_ptr<double>(ws, lay.off_q);
    HIPCHK(hipMemcpyAsync(d_nusf, nusf, mg * 8, hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(d_chi, chi, mg * 8, hipMemcpyHostToDevice, stream));
    int rc = reset();
    if (rc) return rc;
    const FsrArgs f = fsr_args();
    const size_t nfg = (size_t)f.n;
    k_fill_f64<<<(unsigned)std::min<size_t>((nfg + 255) / 256, 65536), 256, 0, stream>>>(f.phi, 1.0, nfg);
    HIPCHK(hipGetLastError());
    has_source = true;
    const long long nfsr = info.n_fsr;
    const unsigned fb = (unsigned)((nfg + 255) / 256), jb = (unsigned)((nfsr + 255) / 256);
    std::vector<double> sl((size_t)kSlots * kSlotStride * 3);
    // the three eigenvalue quantities sit next to each other in the scalar block
    const size_t s0 = slot_index(Q_PNEW, 0);
    auto read_slots = [&]() -> int {
        HIPCHK(hipMemcpyAsync(sl.data(), ws + lay.off_scal + s0 * 8, sl.size() * 8, hipMemcpyDeviceToHost,
                              stream));
        HIPCHK(hipStreamSynchronize(stream));
        return MOC_OK;
    };
    auto slot = [&](int q, int i) { return sl[slot_index(q, i) - s0]; };
    double k = 1.0, res = 1.0;
    int it = 0;
    for (it = 1; it <= o.max_iters; ++it) {
        k_fission_source<<<fb, 256, 0, stream>>>(f, d_q, d_nusf, d_chi, 1.0 / k, d_fold);
        HIPCHK(hipGetLastError());
        rc = iterate(1, o, true);
        if (rc) return rc;
        k_production<<<jb, 256, 0, stream>>>(f, d_nusf, d_fold);
        HIPCHK(hipGetLastError());
        if ((rc = read_slots())) return rc;
        double pn = 0.0, po = 0.0;
        for (int i = 0; i < kSlots; ++i) {
            pn += slot(Q_PNEW, i);
            po += slot(Q_POLD, i);
        }
        if (!(po > 0.0) || !(pn > 0.0)) {
            set_error("no fission production: nu_sigma_f is zero wherever there is flux");
            return MOC_EINVAL;
        }
        const double kn = k * pn / po;
        k_shape_residual<<<jb, 256, 0, stream>>>(f, d_nusf, d_fold, po / pn);
        HIPCHK(hipGetLastError());
        if ((rc = read_slots())) return rc;
        double shape = 0.0;
        for (int i = 0; i < kSlots; ++i) shape = std::max(shape, slot(Q_SHAPE, i));
        res = (it == 1) ? 1.0 : std::max(shape, std::fabs(kn - k) / std::fabs(kn));
        k = kn;
        if (it > 1 && res < o.tol) break;
    }
    *k_out = k;
    *res_out = res;
    *iters_out = std::min(it, o.max_iters);
    return MOC_OK;
}

int Solver::read_residual(double *r) {
    // the Q_RES slots are one contiguous run of kSlots * kSlotStride doubles
    std::vector<double> sl((size_t)kSlots * kSlotStride);
    HIPCHK(hipMemcpyAsync(sl.data(), ws + lay.off_scal + slot_index(Q_RES, 0) * 8, sl.size() * 8,
                          hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    double m = 0.0;
    for (int i = 0; i < kSlots; ++i) m = std::max(m, sl[(size_t)i * kSlotStride]);
    *r = (iter <= 1) ? 1.0 : m;
    return MOC_OK;
}

int Solver::sweep_items(long long n_items, const long long *items, const double *qhat,
                        const double *psi_in, int fp64, double *acc_out, double *psi_out) {
    if (chain_only) {
        set_error("a chain-only solver has no boundary buffer for the test hooks");
        return MOC_EINVAL;
    }
    const int G = info.n_groups, T = info.tracks_per_wave;
    const long long nfg = (long long)info.n_fsr * G;
    // staging inside the workspace: items, entry and exit flux per (item, lane)
    const size_t cap = lay.n_item_cap;
    char *it_buf = ws + lay.off_items;
    double *entry = ws_ptr<double>(ws, lay.off_psi_entry);
    double *exitb = ws_ptr<double>(ws, lay.off_psi_exitb);
    std::vector<double> q64(qhat, qhat + nfg);
    std::vector<float> q32(q64.begin(), q64.end());
    HIPCHK(hipMemcpyAsync(ws + lay.off_qhat64, q64.data(), nfg * 8, hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(ws + lay.off_qhat32, q32.data(), nfg * 4, hipMemcpyHostToDevice, stream));
    int rc = fill_zero(ws + lay.off_acc, nfg * 8, stream);
    if (!rc) rc = fill_zero(ws + lay.off_scal, 128 * 1024, stream);
    if (!rc) rc = fill_zero(ws + lay.off_psi0, lay.psi_bytes, stream);
    if (rc) return rc;
    const bool windowed = window_size(fp64 != 0) >= 1;
    std::vector<double> ent, ex;
    std::vector<int> units, fn;
    std::vector<long long> fi0;
    for (long long b = 0; b < n_items; b += (long long)cap) {
        const long long nb = std::min<long long>(cap, n_items - b);
        ent.assign(nb * kItemStride, 0.0);
        for (long long w = 0; w < nb; ++w)
            for (int tr = 0; tr < T; ++tr)
                for (int g = 0; g < G; ++g)
                    ent[w * kItemStride + tr * G + g] = psi_in[((b + w) * T + tr) * G + g];
        HIPCHK(hipMemcpyAsync(entry, ent.data(), nb * kItemStride * 8, hipMemcpyHostToDevice, stream));
        SweepArgs a = sweep_args(fp64, 0);
        a.psi_in = ws + lay.off_psi0;      // scratch for flux carried between windows
        a.psi_out = nullptr;
        a.psi_entry = entry;
        a.psi_exit = exitb;
        if (windowed) {
            // item (2*chunk + dir) -> unit (2D track, dir) restricted to the
            // chunk's polar stack and lines
            units.assign(nb, 0);
            fn.assign(nb, 0);
            fi0.assign(nb, 0);
            for (long long w = 0; w < nb; ++w) {
                const long long item = items[b + w], chunk = item >> 1;
                const long long st = std::upper_bound(chunk_off.begin(), chunk_off.end(), chunk) -
                                     chunk_off.begin() - 1;
                units[w] = (int)(2 * (st / P) + (item & 1));
                fn[w] = (int)(st % P);
                fi0[w] = (chunk - chunk_off[st]) * T;
            }
            HIPCHK(hipMemcpyAsync(ws + lay.off_units, units.data(), nb * 4, hipMemcpyHostToDevice, stream));
            HIPCHK(hipMemcpyAsync(ws + lay.off_filt_n, fn.data(), nb * 4, hipMemcpyHostToDevice, stream));
            HIPCHK(hipMemcpyAsync(ws + lay.off_filt_i0, fi0.data(), nb * 8, hipMemcpyHostToDevice, stream));
            launch_sweep(a, fp64 != 0, ws_ptr<int>(ws, lay.off_units), (int)nb,
                         ws_ptr<int>(ws, lay.off_filt_n), ws_ptr<long long>(ws, lay.off_filt_i0));
        } else {
            HIPCHK(hipMemcpyAsync(it_buf, items + b, nb * 8, hipMemcpyHostToDevice, stream));
            a.items = (const long long *)it_buf;
            a.n_items = nb;
            launch_sweep(a, fp64 != 0);
        }
        HIPCHK(hipGetLastError());
        ex.assign(nb * kItemStride, 0.0);
        HIPCHK(hipMemcpyAsync(ex.data(), exitb, nb * kItemStride * 8, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        for (long long w = 0; w < nb; ++w)
            for (int tr = 0; tr < T; ++tr)
                for (int g = 0; g < G; ++g)
                    psi_out[((b + w) * T + tr) * G + g] = ex[w * kItemStride + tr * G + g];
    }
    HIPCHK(hipMemcpyAsync(acc_out, ws + lay.off_acc, nfg * 8, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    return reset();
}

int Solver::gather_boundary(long long n, const long long *slots, double *out) {
    if (chain_only) {
        set_error("a chain-only solver has no boundary buffers");
        return MOC_EINVAL;
    }
    if (n <= 0) return MOC_OK;
    const int G = info.n_groups;
    // the buffer the next iteration reads: psi0 after an even number of iterations
    const char *buf = ws + ((iter % 2 == 0) ? lay.off_psi0 : lay.off_psi1);
    // staging in the test-hook scratch: slot ids in the entry region, values in the exit region
    const long long per = (long long)(lay.n_item_cap * kItemStride) / G;
    long long *d_slots = ws_ptr<long long>(ws, lay.off_psi_entry);
    double *d_out = ws_ptr<double>(ws, lay.off_psi_exitb);
    for (long long b = 0; b < n; b += per) {
        const long long nb = std::min(per, n - b);
        HIPCHK(hipMemcpyAsync(d_slots, slots + b, nb * 8, hipMemcpyHostToDevice, stream));
        const unsigned blocks = (unsigned)((nb * G + 255) / 256);
        if (lay.psi64) k_gather_slots<double><<<blocks, 256, 0, stream>>>((const double *)buf, d_slots, nb, G, d_out);
        else k_gather_slots<float><<<blocks, 256, 0, stream>>>((const float *)buf, d_slots, nb, G, d_out);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(out + b * G, d_out, (size_t)nb * G * 8, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
    }
    return MOC_OK;
}

int Solver::trace_tracks(long long n, const long long *ids, int cap, int *fsr, double *len,
                         int *count) {
    const long long per = std::max<long long>(
        1, std::min<long long>(1024, (long long)((lay.scratch_bytes - 1024) / ((size_t)cap * 12 + 16))));
    char *sb = ws + lay.off_items;
    for (long long b = 0; b < n; b += per) {
        const long long nb = std::min(per, n - b);
        long long *d_ids = (long long *)sb;
        int *d_cnt = (int *)(sb + ((nb * 8 + 255) & ~255LL));
        double *d_len = (double *)((char *)d_cnt + ((nb * 4 + 255) & ~255LL));
        int *d_fsr = (int *)((char *)d_len + (((size_t)nb * cap * 8 + 255) & ~size_t(255)));
        HIPCHK(hipMemcpyAsync(d_ids, ids + b, nb * 8, hipMemcpyHostToDevice, stream));
        SweepArgs a = sweep_args(0, 0);
        k_trace<<<(unsigned)((nb + 63) / 64), 64, 0, stream>>>(a, d_ids, nb, cap, d_fsr, d_len,
                                                                 d_cnt);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(count + b, d_cnt, nb * 4, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipMemcpyAsync(fsr + b * cap, d_fsr, (size_t)nb * cap * 4, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipMemcpyAsync(len + b * cap, d_len, (size_t)nb * cap * 8, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
    }
    return MOC_OK;
}

}  // namespace moc
