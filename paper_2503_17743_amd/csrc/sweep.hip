// gfx950 kernels of one fixed-source 3D MOC source iteration:
//   source update -> on-the-fly 3D segment generation + Eq. 3 sweep + FSR
//   tally + boundary angular-flux exchange -> finalize (Eq. 4 estimator,
//   residual, balance).
//
// Sweep mapping.  One wavefront (64 lanes) takes a bundle of T = 64/G
// consecutive lines of one z-stack (paper Eq. 5: same 2D track, same polar
// angle, dz apart) in one sweep direction; lane = (line in bundle, group).
// All lines of a bundle project onto the same 2D track, so the wave walks
// that track's 2D segments in lockstep (uniform loop, the segment record is
// shared by the whole wave) and every lane splits the current 2D segment at
// the axial planes it crosses (Eqs. 6-11 evaluated per line: a line inside one
// layer over the whole 2D segment has length ds/sin(theta) (Eq. 8), a line
// crossing a whole layer has length dz_layer/|cos(theta)| (Eq. 11)).  3D
// segments live only in registers: nothing per 3D track or segment is stored.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "plan.hpp"
#include "solver.hpp"

namespace moc {

constexpr double kFourPi = 12.566370614359172953850573533118;
constexpr int kSlots = 64;        // spread of the scalar accumulators
constexpr int kSlotStride = 16;   // doubles between slots (separate cache lines)

// scalar accumulator layout inside the scalar block (doubles / u64)
enum ScalarQ { Q_SIN = 0, Q_SOUT, Q_LEAK, Q_NSEG, Q_LINKERR, Q_BAL, Q_ABS, Q_SRC, Q_COUNT };
__host__ __device__ inline size_t slot_index(int q, int slot) {
    return 64 + ((size_t)q * kSlots + slot) * kSlotStride;
}

// ------------------------------------------------------------------ helpers

template <typename R>
__device__ inline R one_minus_exp(R tau, int exp_mode);

template <>
__device__ inline float one_minus_exp<float>(float tau, int exp_mode) {
    // stable 1 - e^{-tau}: expm1 keeps full relative accuracy for small tau
    if (exp_mode == 0) return -expm1f(-tau);
    return 1.0f - __expf(-tau);
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

__device__ inline void clip_line(double base, double c, double Lt, double H, double &ls,
                                 double &le) {
    double a, b;
    if (c > 0) {
        a = -base / c;
        b = (H - base) / c;
    } else {
        a = (H - base) / c;
        b = -base / c;
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

// ------------------------------------------------------------------ sweep

struct SweepArgs {
    const double *cot, *secl, *seca, *wgt;       // [A2][P]
    const double *t_len;                          // [n2d]
    const int *t_first, *t_meta, *t_link;         // [n2d+1], [n2d], [2*n2d]
    const double *seg_pos;                        // [nseg]
    const int *seg_reg, *reg_mat;                 // [nseg], [n_regions]
    const double *zeta;                           // [n_stacks]
    const long long *ilo;                         // [n_stacks]
    const int *cnt;                               // [n_stacks]
    const long long *trk_off, *chunk_off;         // [n_stacks+1]
    const void *sigt;                             // [M][G] float or double
    const void *qhat;                             // [n_fsr][G] float or double
    double *acc;                                  // [n_fsr][G]
    const void *psi_in;                           // boundary buffer read this sweep
    void *psi_out;                                // boundary buffer written (may be null)
    const double *psi_entry;                      // per (wave, lane) incoming flux (test hook)
    double *psi_exit;                             // per (wave, lane) outgoing flux (test hook)
    const long long *items;                       // explicit work list or null
    long long n_items;
    long long n_stacks;
    double *scal;
    double H, h, dz;
    int G, P, K, T;
    int bc[6];
    int exp_mode;
    int mode;                                     // 0 sweep, 1 volume tally
};

// One wave = one work item (2*chunk + dir).  Lanes beyond T*G or beyond the
// stack's line count are inactive but follow the uniform loops.  R is the
// segment arithmetic type, B the storage type of the boundary flux.
template <typename R, typename B>
__global__ __launch_bounds__(256) void k_sweep(SweepArgs a) {
    const int lane = threadIdx.x & 63;
    const long long w = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (w >= a.n_items) return;
    const long long item = a.items ? a.items[w] : w;
    const int dir = (int)(item & 1);
    const long long chunk = item >> 1;
    // stack of this chunk: largest s with chunk_off[s] <= chunk
    long long lo = 0, hi = a.n_stacks;
    while (hi - lo > 1) {
        long long mid = (lo + hi) >> 1;
        if (a.chunk_off[mid] <= chunk) lo = mid;
        else hi = mid;
    }
    const long long s = lo;
    const int P = a.P, G = a.G, K = a.K;
    const long long t = s / P;
    const int n = (int)(s - t * P);
    const int meta = a.t_meta[t];
    const int az = meta & 0xffff;
    const int an = az * P + n;
    const double c = a.cot[an];
    const double secl = a.secl[an];     // 3D length per unit 2D length (1/sin)
    const double seca = a.seca[an];     // 3D length per unit height (1/|cos|)
    const double W = a.wgt[an];
    const double Lt = a.t_len[t];
    const int f0 = a.t_first[t], f1 = a.t_first[t + 1];
    const int tr = lane / G;
    const int g = lane - tr * G;
    const long long zi = (chunk - a.chunk_off[s]) * a.T + tr;
    const bool active = (tr < a.T) && (zi < (long long)a.cnt[s]);
    const double base = a.zeta[s] + (double)(a.ilo[s] + zi) * a.dz;
    double ls = 1e300, le = -1e300;
    if (active) clip_line(base, c, Lt, a.H, ls, le);
    const double l_lo = wave_min(ls), l_hi = wave_max(le);
    const long long slot_in = 2 * (a.trk_off[s] + zi) + dir;

    const R *sigt = (const R *)a.sigt;
    const R *qhat = (const R *)a.qhat;
    R psi = 0;
    if (active) {
        if (a.psi_entry) psi = (R)a.psi_entry[w * 64 + lane];
        else if (a.mode == 0) psi = (R)((const B *)a.psi_in)[slot_in * G + g];
    }
    const double psi_start = (double)psi;
    long long nseg = 0;

    const int k_first = seg_search(a.seg_pos, f0, f1, l_lo);
    const int k_last = seg_search(a.seg_pos, f0, f1, l_hi);
    const bool up = (c > 0) != (dir == 1);   // vertical motion in sweep order
    const int nk = k_last - k_first + 1;
    for (int kk = 0; kk < nk; ++kk) {
        const int k = dir ? (k_last - kk) : (k_first + kk);
        const double s0 = a.seg_pos[k];
        const double s1 = (k + 1 < f1) ? a.seg_pos[k + 1] : Lt;
        const int reg = a.seg_reg[k];
        const long long jb = (long long)reg * K;
        if (!active) continue;
        const double sa = fmax(s0, ls), sb = fmin(s1, le);
        if (!(sa < sb)) continue;
        const R st = (g < G) ? sigt[a.reg_mat[reg] * G + g] : (R)0;
        const double za = base + c * sa, zb = base + c * sb;
        const double zlo = fmin(za, zb), zhi = fmax(za, zb);
        int kl = (int)floor(zlo / a.h), kh = (int)ceil(zhi / a.h) - 1;
        kl = min(max(kl, 0), K - 1);
        kh = min(max(kh, kl), K - 1);
        const int np = kh - kl + 1;
        for (int p = 0; p < np; ++p) {
            const int kz = up ? kl + p : kh - p;
            double l3;
            if (np == 1) {
                l3 = (sb - sa) * secl;                         // Eq. 8 case
            } else {
                const double zl = fmax(zlo, kz * a.h), zh = fmin(zhi, (kz + 1) * a.h);
                l3 = (zh - zl) * seca;                         // Eq. 11 / partial
            }
            if (!(l3 >= kMinSeg)) continue;
            const long long j = jb + kz;
            ++nseg;
            if (a.mode == 1) {
                if (g == 0) unsafeAtomicAdd(&a.acc[j], W * l3 / kFourPi);
                continue;
            }
            const R q = qhat[j * G + g];
            const R F = one_minus_exp<R>(st * (R)l3, a.exp_mode);
            const R d = (psi - q) * F;                         // Eq. 3
            psi -= d;
            unsafeAtomicAdd(&a.acc[j * G + g], W * (double)d);
        }
    }
    if (a.mode == 1) {
        const long long tot = wave_sum_ll(active && g == 0 ? nseg : 0);
        if (lane == 0) atomicAdd((unsigned long long *)&a.scal[slot_index(Q_NSEG, (int)(w % kSlots))],
                                 (unsigned long long)tot);
        return;
    }

    // ---- boundary angular flux: hand psi to the directed track that starts
    // where this one leaves the box (specular reflection), or leak it.
    double leak = 0.0;
    long long link_err = 0;
    if (active) {
        if (a.psi_exit) a.psi_exit[w * 64 + lane] = (double)psi;
        const double zf = up ? a.H : 0.0;
        const int face_z = up ? MOC_FACE_ZMAX : MOC_FACE_ZMIN;
        const double lf = (zf - base) / c;       // where the line meets that face
        int kind;                                 // 0 z-face, 1 side, 2 edge
        if (dir == 0) kind = (lf < Lt - kTrackEps) ? 0 : (lf > Lt + kTrackEps) ? 1 : 2;
        else kind = (lf > kTrackEps) ? 0 : (lf < -kTrackEps) ? 1 : 2;
        const int face_s = dir == 0 ? ((meta >> 20) & 0xf) : ((meta >> 16) & 0xf);
        bool vac = false;
        if (kind != 1) vac |= (a.bc[face_z] == MOC_BC_VACUUM);
        if (kind != 0) vac |= (a.bc[face_s] == MOC_BC_VACUUM);
        if (vac) {
            leak = W * (double)psi;
        } else if (a.psi_out) {
            long long t2;
            int d2, n2;
            double l2, z2;
            if (kind == 0) {
                t2 = t;
                d2 = dir;
                n2 = P - 1 - n;
                l2 = lf;
                z2 = zf;
            } else {
                const int lk = a.t_link[2 * t + dir];
                t2 = lk >> 1;
                d2 = lk & 1;
                const bool same = (d2 == dir);
                n2 = (kind == 1) == same ? n : P - 1 - n;
                l2 = d2 == 0 ? 0.0 : a.t_len[t2];
                z2 = kind == 1 ? base + c * (dir == 0 ? Lt : 0.0) : zf;
            }
            const long long s2 = t2 * P + n2;
            const int an2 = (a.t_meta[t2] & 0xffff) * P + n2;
            const double c2 = a.cot[an2];
            const long long i2 =
                llrint((z2 - a.zeta[s2] - c2 * l2) / a.dz) - a.ilo[s2];
            if (i2 >= 0 && i2 < (long long)a.cnt[s2]) {
                const long long slot2 = 2 * (a.trk_off[s2] + i2) + d2;
                ((B *)a.psi_out)[slot2 * G + g] = (B)psi;
            } else {
                link_err = 1;
                leak = W * (double)psi;
            }
        }
    }
    const double sin_ = wave_sum(active ? W * psi_start : 0.0);
    const double sout = wave_sum(active ? W * (double)psi : 0.0);
    const double lk = wave_sum(leak);
    const long long ns = wave_sum_ll(active ? nseg : 0);
    const long long le_ = wave_sum_ll(link_err);
    if (lane == 0) {
        const int sl = (int)(w % kSlots);
        unsafeAtomicAdd(&a.scal[slot_index(Q_SIN, sl)], sin_);
        unsafeAtomicAdd(&a.scal[slot_index(Q_SOUT, sl)], sout);
        unsafeAtomicAdd(&a.scal[slot_index(Q_LEAK, sl)], lk);
        atomicAdd((unsigned long long *)&a.scal[slot_index(Q_NSEG, sl)], (unsigned long long)ns);
        if (le_) atomicAdd((unsigned long long *)&a.scal[slot_index(Q_LINKERR, sl)], (unsigned long long)le_);
    }
}

// ------------------------------------------------------------------ trace hook

// One thread per requested stored track (forward): the same per-2D-segment
// axial splitting as the sweep, written out instead of swept.
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
    const double c = a.cot[an], secl = a.secl[an], seca = a.seca[an];
    const double Lt = a.t_len[t];
    const int f0 = a.t_first[t], f1 = a.t_first[t + 1];
    const long long zi = trk - a.trk_off[s];
    const double base = a.zeta[s] + (double)(a.ilo[s] + zi) * a.dz;
    double ls, le;
    clip_line(base, c, Lt, a.H, ls, le);
    const bool up = c > 0;
    int m = 0;
    for (int k = seg_search(a.seg_pos, f0, f1, ls); k < f1; ++k) {
        const double s0 = a.seg_pos[k];
        if (s0 >= le) break;
        const double s1 = (k + 1 < f1) ? a.seg_pos[k + 1] : Lt;
        const double sa = fmax(s0, ls), sb = fmin(s1, le);
        if (!(sa < sb)) continue;
        const double za = base + c * sa, zb = base + c * sb;
        const double zlo = fmin(za, zb), zhi = fmax(za, zb);
        int kl = (int)floor(zlo / a.h), kh = (int)ceil(zhi / a.h) - 1;
        kl = min(max(kl, 0), K - 1);
        kh = min(max(kh, kl), K - 1);
        const int np = kh - kl + 1;
        for (int p = 0; p < np; ++p) {
            const int kz = up ? kl + p : kh - p;
            double l3;
            if (np == 1) l3 = (sb - sa) * secl;
            else {
                const double zl = fmax(zlo, kz * a.h), zh = fmin(zhi, (kz + 1) * a.h);
                l3 = (zh - zl) * seca;
            }
            if (!(l3 >= kMinSeg)) continue;
            if (m < cap) {
                fsr[i * cap + m] = (int)((long long)a.seg_reg[k] * K + kz);
                len[i * cap + m] = l3;
            }
            ++m;
        }
    }
    count[i] = m;
}

// ------------------------------------------------------------------ source / finalize

struct FsrArgs {
    const double *q, *sigt, *sigs, *vol;
    const int *reg_mat;
    double *phi, *acc, *qhat64;
    float *qhat32;
    double *scal;
    long long n;        // n_fsr * G
    int G, K;
};

// qhat = (sum_g' Sigma_s[g'->g] phi_g' + Q_g) / (4 pi Sigma_t,g); clears the tally.
__global__ __launch_bounds__(256) void k_source(FsrArgs a) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
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
__global__ __launch_bounds__(256) void k_finalize(FsrArgs a) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
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
    res = wave_max(res);
    bal = wave_sum(bal);
    absb = wave_sum(absb);
    src = wave_sum(src);
    if ((threadIdx.x & 63) == 0) {
        const int sl = (int)(((long long)blockIdx.x * 4 + (threadIdx.x >> 6)) % kSlots);
        atomicMax((unsigned long long *)&a.scal[0], (unsigned long long)__double_as_longlong(res));
        unsafeAtomicAdd(&a.scal[slot_index(Q_BAL, sl)], bal);
        unsafeAtomicAdd(&a.scal[slot_index(Q_ABS, sl)], absb);
        unsafeAtomicAdd(&a.scal[slot_index(Q_SRC, sl)], src);
    }
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
    a.seca = ws_ptr<double>(ws, lay.off_seca);
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
    a.qhat = fp64 ? (const void *)ws_ptr<double>(ws, lay.off_qhat64)
                  : (const void *)ws_ptr<float>(ws, lay.off_qhat32);
    a.acc = ws_ptr<double>(ws, lay.off_acc);
    a.scal = ws_ptr<double>(ws, lay.off_scal);
    a.n_items = 2 * info.n_chunks;
    a.n_stacks = info.n_stacks;
    a.H = H;
    a.h = h;
    a.dz = info.dz;
    a.G = info.n_groups;
    a.P = P;
    a.K = K;
    a.T = info.tracks_per_wave;
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
    std::vector<double> secl(p.cot.size()), seca(p.cot.size());
    for (size_t i = 0; i < p.cot.size(); ++i) {
        double c = p.cot[i];
        secl[i] = std::sqrt(1.0 + c * c);
        seca[i] = std::sqrt(1.0 + c * c) / std::fabs(c);
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
    HIPCHK(put(lay.off_seca, seca.data(), seca.size() * 8));
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
    HIPCHK(put(lay.off_sigt32, sigt32.data(), sigt32.size() * 4));
    HIPCHK(put(lay.off_sigt64, p.sigt.data(), p.sigt.size() * 8));
    HIPCHK(put(lay.off_sigs, p.sigs.data(), p.sigs.size() * 8));
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

void Solver::launch_sweep(const SweepArgs &a, bool fp64) {
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

int Solver::reset() {
    int rc = fill_zero(ws + lay.off_phi, (size_t)info.n_fsr * info.n_groups * 8, stream);
    if (!rc) rc = fill_zero(ws + lay.off_psi0, lay.psi_bytes, stream);
    iter = 0;
    sweep_ms.clear();
    return rc;
}

int Solver::iterate(int nit, const moc_solve_opts &o, bool time_sweep) {
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
        int rc = fill_zero(ws + lay.off_scal, 128 * 1024, stream);
        if (rc) return rc;
        k_source<<<fblocks, 256, 0, stream>>>(f);
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

Solver::~Solver() {
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
    st->residual = (iter <= 1) ? 1.0 : sc[0];
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

int Solver::read_residual(double *r) {
    HIPCHK(hipMemcpyAsync(r, ws + lay.off_scal, 8, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    if (iter <= 1) *r = 1.0;
    return MOC_OK;
}

int Solver::sweep_items(long long n_items, const long long *items, const double *qhat,
                        const double *psi_in, int fp64, double *acc_out, double *psi_out) {
    const int G = info.n_groups, T = info.tracks_per_wave;
    const long long nfg = (long long)info.n_fsr * G;
    // staging inside the workspace: items, entry and exit flux per (wave, lane)
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
    if (rc) return rc;
    std::vector<double> ent, ex;
    for (long long b = 0; b < n_items; b += (long long)cap) {
        const long long nb = std::min<long long>(cap, n_items - b);
        ent.assign(nb * 64, 0.0f);
        for (long long w = 0; w < nb; ++w)
            for (int tr = 0; tr < T; ++tr)
                for (int g = 0; g < G; ++g)
                    ent[w * 64 + tr * G + g] = psi_in[((b + w) * T + tr) * G + g];
        HIPCHK(hipMemcpyAsync(it_buf, items + b, nb * 8, hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemcpyAsync(entry, ent.data(), nb * 64 * 8, hipMemcpyHostToDevice, stream));
        SweepArgs a = sweep_args(fp64, 0);
        a.items = (const long long *)it_buf;
        a.n_items = nb;
        a.psi_in = nullptr;
        a.psi_out = nullptr;
        a.psi_entry = entry;
        a.psi_exit = exitb;
        launch_sweep(a, fp64 != 0);
        HIPCHK(hipGetLastError());
        ex.assign(nb * 64, 0.0f);
        HIPCHK(hipMemcpyAsync(ex.data(), exitb, nb * 64 * 8, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        for (long long w = 0; w < nb; ++w)
            for (int tr = 0; tr < T; ++tr)
                for (int g = 0; g < G; ++g)
                    psi_out[((b + w) * T + tr) * G + g] = ex[w * 64 + tr * G + g];
    }
    HIPCHK(hipMemcpyAsync(acc_out, ws + lay.off_acc, nfg * 8, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
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
