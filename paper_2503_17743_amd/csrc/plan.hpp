// Host-side plan of a fixed-source 3D MOC problem: everything the device
// sweep needs that is computed once per problem on the CPU (paper section 3.1:
// geometry modelling and 2D ray tracing stay on the host; 3D tracing and the
// sweep move to the GPU).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/moc.h"

namespace moc {

// A line of a z-stack is a 3D track only if it runs more than this 2D length
// inside the box; lines that merely graze a box edge are not tracks.  The
// same tolerance decides when a track leaves through a box edge.
constexpr double kTrackEps = 1e-9;
// Segments shorter than this (cm) are dropped.  Pieces of zero length in
// exact arithmetic (a layer plane crossed exactly where a radial surface is)
// carry the rounding noise of the chain phase (up to ~1e-11 cm on long
// cycles), far below this; genuine pieces this short are vanishingly rare.
constexpr double kMinSeg = 1e-9;
// Sweep lane layout: the G groups are split into C = ceil(G / kGL) chunks
// across lanes; a lane holds the flux of up to kGL groups in registers and a
// wave bundle covers T = 64 / C lines.
constexpr int kGL = 8;
inline int group_chunks(int G) { return (G + kGL - 1) / kGL; }
inline int groups_per_lane(int G) { return (G + group_chunks(G) - 1) / group_chunks(G); }
// Per-item stride (doubles) of the test hooks' entry/exit flux buffers: T * G
// never exceeds 64 * kGL.
constexpr int kItemStride = 64 * kGL;
// Workgroups of a chain-line sweep (each holds its own carry buffers)
constexpr int kChainSlots = 512;

struct Plan {
    // ---- problem ----
    int nx = 0, ny = 0, ns = 1, K = 1, G = 1, M = 1, P = 2, A = 4, A2 = 2, A4 = 1, Rc = 1;
    double pitch = 1, R = 0, H = 1, Wx = 1, Wy = 1, h = 1, dz = 1;
    int bc[6] = {0, 0, 0, 0, 0, 0};
    std::vector<int> cell_mat;            // [ncell][2]
    std::vector<double> sigt, sigs;       // [M][G], [M][G][G]
    int64_t n_regions = 0, n_fsr = 0;

    // ---- quadrature (stored azimuths a in [0, A/2)) ----
    std::vector<double> phi, dphi, deff, LC;   // [A2]
    std::vector<int> nxa, nya;                 // [A2]
    std::vector<double> mu, wp;                // [P]
    std::vector<double> cot, wgt;              // [A2][P]

    // ---- 2D tracks ----
    int64_t n2d = 0;
    std::vector<double> x0, y0, x1, y1, L, chain;
    std::vector<int> az, face0, face1, sig;
    std::vector<int64_t> link;                 // [2*n2d] successor directed id 2*t+d
    std::vector<int64_t> seg_first;            // [n2d+1]

    // ---- 2D segments ----
    std::vector<double> seg_pos;               // start position along the 2D track
    std::vector<int> seg_reg;                  // radial region

    std::vector<int> reg_mat;                  // [n_regions]

    // ---- z-stacks (s = t*P + n) ----
    int64_t n_stacks = 0, n3d = 0, n_chunks = 0;
    int T = 1;                                 // tracks per wave (bundle size)
    int lstride = 1;                           // line stride inside a bundle
    std::vector<double> zeta;
    std::vector<int64_t> ilo, cnt, trk_off, chunk_off;   // trk_off/chunk_off: [n_stacks+1]

    // ---- chain-line sweep (vacuum top and bottom faces only) ----
    // A traversal is a directed 2D cycle, its units (2*t + dir) in link order
    // from the cycle's chain origin.  Each traversal is cut into segments:
    // segment k of K takes, for every polar angle, the lines entering the box
    // (rising through the bottom face, falling through the top one) within
    // [A_k, A_{k+1}) of the traversal's length, A_k a whole number of that
    // angle's entry spacings L_C / kk (kk lines cross a point per cycle).  Its
    // items are the units those lines cross, in traversal order, with each
    // unit's unrolled start (its start plus whole traversal lengths once the
    // lines wrap past the origin).  Segments are listed longest first.
    int64_t n_trav = 0, n_chseg = 0;
    std::vector<int> ch_first;                 // [n_chseg+1] item range of each segment
    std::vector<int> ch_code;                  // [items] unit code
    std::vector<double> ch_u;                  // [items] unrolled start of the unit
    std::vector<int> ch_k, ch_nk;              // [n_chseg] segment index, segments of its traversal
    std::vector<double> ch_lc;                 // [n_chseg] length of its traversal
    int64_t ch_cap = 0;                        // lines of the largest stack

    std::string build(const moc_geometry &g, const moc_tracking &t, const moc_xs &x);
    moc_plan_info info() const;
};

// Device layout of a plan inside a caller workspace.
struct Layout {
    size_t total = 0;
    size_t off_cot = 0, off_secl = 0, off_icot = 0, off_wgt = 0;  // [A2][P] doubles
    size_t off_t_len = 0, off_t_first = 0, off_t_meta = 0, off_t_link = 0;
    size_t off_seg_pos = 0, off_seg_reg = 0, off_reg_mat = 0;
    size_t off_seg_st = 0;          // [nseg][G] float: Sigma_t log2(e) per 2D segment
    size_t off_zeta = 0, off_ilo = 0, off_cnt = 0, off_trk_off = 0, off_chunk_off = 0;
    size_t off_sigt32 = 0, off_sigt64 = 0, off_sigs = 0;
    size_t off_q = 0, off_qhat32 = 0, off_qhat64 = 0, off_acc = 0, off_phi = 0, off_vol = 0;
    size_t off_psi0 = 0, off_psi1 = 0, psi_bytes = 0;
    size_t off_scal = 0;
    // eigenvalue mode: nu Sigma_f and chi [M][G], fission production of the
    // previous iterate [n_fsr]
    size_t off_nusf = 0, off_chi = 0, off_fold = 0;
    // scratch for the test hooks: work list + entry/exit flux per (wave, lane);
    // the same region holds traced segments
    size_t off_items = 0, off_psi_entry = 0, off_psi_exitb = 0;
    size_t off_units = 0, off_filt_n = 0, off_filt_i0 = 0;
    size_t n_item_cap = 0, scratch_bytes = 0;
    size_t off_work = 0;            // windowed-sweep work list (2 * n2d codes)
    size_t off_ch_first = 0, off_ch_code = 0, off_ch_u = 0, off_ch_k = 0, off_ch_nk = 0, off_ch_lc = 0;
    size_t off_ch_ctr = 0;          // next segment to take (reset before each chain sweep)
    // chain sweep carry buffers: per workgroup (kChainSlots at most) two
    // parities x P stacks x ch_cap lines x G fluxes of the boundary type
    size_t off_ch_carry = 0;
    bool psi64 = false;             // boundary angular flux stored in FP64
};

Layout make_layout(const Plan &p, bool psi64);

}  // namespace moc

struct moc_plan {
    moc::Plan p;
};
