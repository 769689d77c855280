// Host planner: quadrature, cyclic 2D laydown, 2D ray tracing of the radial
// geometry, reflective cycles with chain phases, and the z-stack table.
//
// Paper anchors: section 3.1 (2D ray tracing on the CPU, data copied to the
// GPU), section 2.2 (axially extruded geometry: only 2D segments are stored;
// Eq. 5 places the lines of a z-stack), section 3.2 / Eq. 13 (the z-stack
// table flattened as stack[z[i] + j*c + k]).  The quadrature, the laydown
// and the chain phase are readings of points the paper leaves open; they are
// restated in the comments below.
#include "plan.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <tuple>

namespace moc {

namespace {

constexpr double kPi = 3.14159265358979323846;

// Gauss-Legendre nodes (ascending) and weights by Newton iteration on the
// Legendre recurrence; the positive half is computed and mirrored so that the
// rule is exactly symmetric.
void gauss_legendre(int n, std::vector<double> &mu, std::vector<double> &w) {
    mu.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double x = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= n; ++k) {
            double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = pk;
        }
        dp = n * (x * p1 - p0) / (x * x - 1.0);
        double wi = 2.0 / ((1.0 - x * x) * dp * dp);
        mu[n - 1 - i] = x;
        w[n - 1 - i] = wi;
        mu[i] = -x;
        w[i] = wi;
    }
}

int64_t gcd64(int64_t a, int64_t b) {
    while (b) {
        int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// 2D-length interval [ls, le] of line z = base + c*l inside 0<=l<=L, 0<=z<=H
inline void clip(double base, double c, double Lt, double H, double &ls, double &le) {
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

}  // namespace

std::string Plan::build(const moc_geometry &g, const moc_tracking &t, const moc_xs &x) {
    // ------------------------------------------------ validation
    if (t.n_azim < 4 || t.n_azim % 4) return "n_azim must be a positive multiple of 4";
    if (t.n_polar < 2 || t.n_polar % 2) return "n_polar must be even and >= 2";
    if (!(t.radial_spacing > 0) || !(t.axial_spacing > 0)) return "track spacings must be > 0";
    if (g.nx < 1 || g.ny < 1 || !(g.pitch > 0)) return "lattice must be at least 1x1 with pitch > 0";
    if (!(g.height > 0) || g.n_layers < 1) return "height and n_layers must be positive";
    if (g.inclusion_radius < 0 || g.inclusion_radius >= 0.5 * g.pitch)
        return "inclusion radius must be in [0, pitch/2)";
    if (!(g.n_sectors == 1 || g.n_sectors == 2 || g.n_sectors == 4 || g.n_sectors == 8 ||
          g.n_sectors == 16))
        return "n_sectors must be 1, 2, 4, 8 or 16";
    for (int f = 0; f < 6; ++f)
        if (g.bc[f] != MOC_BC_VACUUM && g.bc[f] != MOC_BC_REFLECTIVE) return "bc must be 0 or 1";
    if (x.n_groups < 1 || x.n_groups > 64) return "n_groups must be in [1, 64]";
    if (t.n_polar > 64) return "n_polar must be <= 64";
    if (x.n_materials < 1) return "n_materials must be >= 1";
    if (!g.cell_material || !x.sigma_t || !x.sigma_s) return "null input array";
    nx = g.nx;
    ny = g.ny;
    ns = g.n_sectors;
    K = g.n_layers;
    G = x.n_groups;
    M = x.n_materials;
    P = t.n_polar;
    A = t.n_azim;
    A2 = A / 2;
    A4 = A / 4;
    pitch = g.pitch;
    R = g.inclusion_radius;
    H = g.height;
    Wx = nx * pitch;
    Wy = ny * pitch;
    h = H / K;
    dz = H / std::ceil(H / t.axial_spacing);
    std::memcpy(bc, g.bc, sizeof(bc));
    Rc = (R > 0 ? 2 : 1) * ns;
    n_regions = (int64_t)nx * ny * Rc;
    n_fsr = n_regions * K;
    cell_mat.assign(g.cell_material, g.cell_material + 2 * nx * ny);
    for (int v : cell_mat)
        if (v < 0 || v >= M) return "material id out of range";
    sigt.assign(x.sigma_t, x.sigma_t + (size_t)M * G);
    sigs.assign(x.sigma_s, x.sigma_s + (size_t)M * G * G);
    for (int m = 0; m < M; ++m) {
        for (int gg = 0; gg < G; ++gg) {
            double st = sigt[m * G + gg];
            if (!(st > 0) || !std::isfinite(st)) return "sigma_t must be > 0";
            double out = 0;
            for (int g2 = 0; g2 < G; ++g2) {
                double v = sigs[((size_t)m * G + gg) * G + g2];
                if (!(v >= 0) || !std::isfinite(v)) return "sigma_s must be >= 0";
                out += v;
            }
            if (!(out < st)) return "out-scatter ratio must be < 1";
        }
    }

    // ------------------------------------------------ azimuthal quadrature
    // First quadrant: desired angle 2pi/A (a + 1/2); track counts on the x and
    // y sides; corrected angle atan(Wy nx / (Wx ny)) makes the laydown cyclic;
    // corrected spacing (Wx/nx) sin(phi').  Second quadrant mirrors it.
    phi.assign(A2, 0);
    dphi.assign(A2, 0);
    deff.assign(A2, 0);
    LC.assign(A2, 0);
    nxa.assign(A2, 0);
    nya.assign(A2, 0);
    for (int a = 0; a < A4; ++a) {
        double phid = 2.0 * kPi / A * (a + 0.5);
        nxa[a] = (int)std::ceil(Wx / t.radial_spacing * std::fabs(std::sin(phid)));
        nya[a] = (int)std::ceil(Wy / t.radial_spacing * std::fabs(std::cos(phid)));
        phi[a] = std::atan((Wy * nxa[a]) / (Wx * nya[a]));
        deff[a] = (Wx / nxa[a]) * std::sin(phi[a]);
    }
    for (int a = A4; a < A2; ++a) {
        int am = A2 - 1 - a;
        nxa[a] = nxa[am];
        nya[a] = nya[am];
        phi[a] = kPi - phi[am];
        deff[a] = deff[am];
    }
    // azimuthal weight: half the angular gap between neighbouring corrected
    // angles, with the quadrant edges reflected
    for (int a = 0; a < A4; ++a) {
        double prev = (a == 0) ? -phi[0] : phi[a - 1];
        double next = (a == A4 - 1) ? kPi - phi[A4 - 1] : phi[a + 1];
        dphi[a] = 0.5 * (next - prev);
        dphi[A2 - 1 - a] = dphi[a];
    }
    // length of one reflective cycle of an azimuth pair
    for (int a = 0; a < A2; ++a) {
        double gg = (double)gcd64(nxa[a], nya[a]);
        double lx = 2.0 * Wx * nya[a] / gg, ly = 2.0 * Wy * nxa[a] / gg;
        LC[a] = std::sqrt(lx * lx + ly * ly);
    }

    // ------------------------------------------------ polar quadrature
    // Gauss-Legendre in mu = cos(theta); per azimuth the cotangent is rounded
    // to an integer number k of axial spacings per cycle (cot = k dz / L_C) so
    // that every z-stack line closes on itself after one cycle.
    gauss_legendre(P, mu, wp);
    cot.assign((size_t)A2 * P, 0);
    wgt.assign((size_t)A2 * P, 0);
    for (int a = 0; a < A2; ++a) {
        for (int n = P / 2; n < P; ++n) {
            double c0 = mu[n] / std::sqrt(1.0 - mu[n] * mu[n]);
            double kk = std::floor(LC[a] * c0 / dz + 0.5);
            if (kk < 1) kk = 1;
            double c = kk * dz / LC[a];
            cot[a * P + n] = c;
            cot[a * P + (P - 1 - n)] = -c;
        }
        for (int n = 0; n < P; ++n) {
            double c = cot[a * P + n];
            double sint = 1.0 / std::sqrt(1.0 + c * c);
            double w = wp[n >= P / 2 ? n : P - 1 - n];
            // solid-angle weight dphi * w times the area one 3D track
            // represents perpendicular to its direction (spacing x dz sin)
            wgt[a * P + n] = dphi[a] * w * deff[a] * dz * sint;
        }
    }

    // ------------------------------------------------ 2D tracks
    n2d = 0;
    for (int a = 0; a < A2; ++a) n2d += nxa[a] + nya[a];
    x0.assign(n2d, 0);
    y0.assign(n2d, 0);
    x1.assign(n2d, 0);
    y1.assign(n2d, 0);
    L.assign(n2d, 0);
    chain.assign(n2d, 0);
    az.assign(n2d, 0);
    face0.assign(n2d, 0);
    face1.assign(n2d, 0);
    sig.assign(n2d, 0);
    link.assign(2 * n2d, -1);
    // boundary point keys: (face, index of the half-offset slot on that face)
    std::vector<std::array<int64_t, 2>> key0(n2d), key1(n2d);
    {
        int64_t tt = 0;
        for (int a = 0; a < A2; ++a) {
            double ux = std::cos(phi[a]), uy = std::sin(phi[a]);
            bool right = a >= A4;
            for (int i = 0; i < nxa[a] + nya[a]; ++i, ++tt) {
                double xs, ys;
                if (i < nxa[a]) {
                    xs = (i + 0.5) * Wx / nxa[a];
                    ys = 0.0;
                    face0[tt] = MOC_FACE_YMIN;
                } else {
                    int j = i - nxa[a];
                    xs = right ? Wx : 0.0;
                    ys = (j + 0.5) * Wy / nya[a];
                    face0[tt] = right ? MOC_FACE_XMAX : MOC_FACE_XMIN;
                }
                double tx = (ux > 0) ? (Wx - xs) / ux : (0.0 - xs) / ux;
                double ty = (Wy - ys) / uy;
                double Lt, xe, ye;
                if (ty < tx) {
                    Lt = ty;
                    xe = xs + Lt * ux;
                    ye = Wy;
                    face1[tt] = MOC_FACE_YMAX;
                } else {
                    Lt = tx;
                    xe = (ux > 0) ? Wx : 0.0;
                    ye = ys + Lt * uy;
                    face1[tt] = (ux > 0) ? MOC_FACE_XMAX : MOC_FACE_XMIN;
                }
                x0[tt] = xs;
                y0[tt] = ys;
                x1[tt] = xe;
                y1[tt] = ye;
                L[tt] = Lt;
                az[tt] = a;
                auto slot = [&](int face, double px, double py) -> int64_t {
                    if (face == MOC_FACE_YMIN || face == MOC_FACE_YMAX)
                        return (int64_t)std::llround(px * nxa[a] / Wx - 0.5);
                    return (int64_t)std::llround(py * nya[a] / Wy - 0.5);
                };
                key0[tt] = {face0[tt], slot(face0[tt], xs, ys)};
                key1[tt] = {face1[tt], slot(face1[tt], xe, ye)};
            }
        }
    }
    // Reflective links by index algebra: on an azimuth pair {a, A2-1-a} every
    // boundary slot is an end point of exactly one track of each azimuth, and
    // specular reflection maps one onto the other.  The successor of a
    // directed track leaves the shared slot along the other track.
    {
        int64_t first = 0;
        std::vector<int64_t> az_first(A2 + 1, 0);
        for (int a = 0; a < A2; ++a) {
            az_first[a] = first;
            first += nxa[a] + nya[a];
        }
        az_first[A2] = first;
        for (int a = 0; a < A4; ++a) {
            int am = A2 - 1 - a;
            // (face, slot) -> list of (track, end) over both azimuths
            std::map<std::pair<int64_t, int64_t>, std::vector<std::pair<int64_t, int>>> pts;
            for (int aa : {a, am})
                for (int64_t tt = az_first[aa]; tt < az_first[aa + 1]; ++tt) {
                    pts[{key0[tt][0], key0[tt][1]}].push_back({tt, 0});
                    pts[{key1[tt][0], key1[tt][1]}].push_back({tt, 1});
                }
            for (auto &kv : pts) {
                if (kv.second.size() != 2) return "internal: cyclic laydown slot not shared by 2 tracks";
                auto e0 = kv.second[0], e1 = kv.second[1];
                if (az[e0.first] == az[e1.first]) return "internal: slot shared within one azimuth";
                // directed track exiting through this slot: (t, fwd) if the slot
                // is its end point, (t, bwd) if it is its start point
                auto exit_id = [](std::pair<int64_t, int> e) { return 2 * e.first + (e.second ? 0 : 1); };
                auto enter_id = [](std::pair<int64_t, int> e) { return 2 * e.first + (e.second ? 1 : 0); };
                link[exit_id(e0)] = enter_id(e1);
                link[exit_id(e1)] = enter_id(e0);
            }
        }
        for (int64_t i = 0; i < 2 * n2d; ++i)
            if (link[i] < 0) return "internal: unlinked 2D track end";
    }
    // Cycles and chain coordinates.  For each pair of mutually reversed
    // directed cycles, C runs the lowest-id track forward; the chain
    // coordinate a_t is measured along C from that track's start point to
    // t's start point, and sigma_t = +1 (-1) when C runs t forward (backward).
    {
        std::vector<char> seen(n2d, 0);
        for (int64_t t0 = 0; t0 < n2d; ++t0) {
            if (seen[t0]) continue;
            int64_t cur = 2 * t0;
            double pos = 0.0;
            int64_t steps = 0;
            do {
                int64_t tt = cur / 2;
                int d = (int)(cur % 2);
                if (seen[tt]) return "internal: cycle equals its reverse";
                seen[tt] = 1;
                if (d == 0) {
                    chain[tt] = pos;
                    sig[tt] = 1;
                } else {
                    chain[tt] = pos + L[tt];
                    sig[tt] = -1;
                }
                pos += L[tt];
                cur = link[cur];
                if (++steps > 2 * n2d) return "internal: cycle does not close";
            } while (cur != 2 * t0);
        }
    }

    // ------------------------------------------------ 2D ray tracing
    // Every crossing of a cell line, inclusion circle and sector half-line
    // along the 2D track is collected, the intervals between them take the
    // region of their midpoint, tiny intervals are dropped and equal
    // neighbours merged.
    reg_mat.assign(n_regions, 0);
    for (int cell = 0; cell < nx * ny; ++cell)
        for (int local = 0; local < Rc; ++local) {
            bool inside = (R > 0) && (local % 2 == 0);
            reg_mat[(int64_t)cell * Rc + local] = cell_mat[2 * cell + (inside ? 0 : 1)];
        }
    auto region_at = [&](double px, double py) -> int {
        int cx = std::min(std::max((int)std::floor(px / pitch), 0), nx - 1);
        int cy = std::min(std::max((int)std::floor(py / pitch), 0), ny - 1);
        double dx = px - (cx + 0.5) * pitch, dy = py - (cy + 0.5) * pitch;
        bool inside = (R > 0) && (dx * dx + dy * dy < R * R);
        int s = 0;
        if (ns > 1) {
            double ang = std::atan2(dy, dx);
            if (ang < 0) ang += 2.0 * kPi;
            // within 1e-9 of a sector line: the sector starting at that line
            s = ((int)std::floor(ang / (2.0 * kPi / ns) + 1e-9)) % ns;
        }
        int local = (R > 0) ? 2 * s + (inside ? 0 : 1) : s;
        return (cy * nx + cx) * Rc + local;
    };
    seg_first.assign(n2d + 1, 0);
    seg_pos.clear();
    seg_reg.clear();
    std::vector<double> ts, cuts;
    for (int64_t tt = 0; tt < n2d; ++tt) {
        double ux = std::cos(phi[az[tt]]), uy = std::sin(phi[az[tt]]);
        double Lt = L[tt];
        cuts.clear();
        for (int k = 1; k < nx; ++k) {
            double s = (k * pitch - x0[tt]) / ux;
            if (s > 0 && s < Lt) cuts.push_back(s);
        }
        for (int k = 1; k < ny; ++k) {
            double s = (k * pitch - y0[tt]) / uy;
            if (s > 0 && s < Lt) cuts.push_back(s);
        }
        std::sort(cuts.begin(), cuts.end());
        ts = cuts;
        if (R > 0 || ns > 1) {
            for (size_t iv = 0; iv <= cuts.size(); ++iv) {
                double sa = iv ? cuts[iv - 1] : 0.0, sb = iv < cuts.size() ? cuts[iv] : Lt;
                double sm = 0.5 * (sa + sb);
                int cx = std::min(std::max((int)std::floor((x0[tt] + sm * ux) / pitch), 0), nx - 1);
                int cy = std::min(std::max((int)std::floor((y0[tt] + sm * uy) / pitch), 0), ny - 1);
                double wx = (cx + 0.5) * pitch - x0[tt], wy = (cy + 0.5) * pitch - y0[tt];
                if (R > 0) {
                    // |p0 + s u - c|^2 = R^2 with |u| = 1
                    double b = wx * ux + wy * uy;
                    double disc = b * b - (wx * wx + wy * wy - R * R);
                    if (disc > 0) {
                        double sq = std::sqrt(disc);
                        for (double r : {b - sq, b + sq})
                            if (r > sa && r < sb) ts.push_back(r);
                    }
                }
                if (ns > 1) {
                    // sector counts are even: every sector boundary is a full
                    // line through the cell centre (half-lines a and a + pi)
                    for (int s = 0; s < ns / 2; ++s) {
                        double al = 2.0 * kPi * s / ns;
                        double ex = std::cos(al), ey = std::sin(al);
                        double den = ux * ey - uy * ex;
                        if (den == 0.0) continue;
                        double sc = (wx * ey - wy * ex) / den;
                        if (sc > sa && sc < sb) ts.push_back(sc);
                    }
                }
            }
        }
        std::sort(ts.begin(), ts.end());
        double prev = 0.0;
        int last = -1;
        for (size_t i = 0; i <= ts.size(); ++i) {
            double s1 = i < ts.size() ? ts[i] : Lt;
            if (s1 - prev >= kMinSeg) {
                double sm = 0.5 * (prev + s1);
                int r = region_at(x0[tt] + sm * ux, y0[tt] + sm * uy);
                if (r != last) {
                    // a new segment starts here (or right after a dropped one)
                    seg_pos.push_back(last < 0 ? 0.0 : prev);
                    seg_reg.push_back(r);
                    last = r;
                }
            }
            prev = s1;
        }
        seg_first[tt + 1] = (int64_t)seg_pos.size();
    }
    if (seg_pos.size() >= (size_t)INT32_MAX) return "too many 2D segments";

    // ------------------------------------------------ z-stacks
    // Eq. 5 with the chain phase: lines z_i(l) = zeta + i dz + l cot, where
    // zeta = dz/2 + sigma_t cot a_t (mod dz).  A stack holds the lines whose
    // intersection with [0, L_t] x [0, H] is longer than kTrackEps.
    n_stacks = n2d * P;
    zeta.assign(n_stacks, 0);
    ilo.assign(n_stacks, 0);
    cnt.assign(n_stacks, 0);
    for (int64_t tt = 0; tt < n2d; ++tt) {
        for (int n = 0; n < P; ++n) {
            int64_t s = tt * P + n;
            double c = cot[az[tt] * P + n];
            double zt = std::fmod(0.5 * dz + sig[tt] * c * chain[tt], dz);
            if (zt < 0) zt += dz;
            if (zt >= dz) zt -= dz;
            zeta[s] = zt;
            auto exists = [&](int64_t i) {
                double ls, le;
                clip(zt + (double)i * dz, c, L[tt], H, ls, le);
                return le - ls > kTrackEps;
            };
            // closed-form bounds, then settle the ends with the same predicate
            double reach = c * L[tt];
            int64_t lo = (c > 0) ? (int64_t)std::ceil(-(zt + reach) / dz) : (int64_t)std::ceil(-zt / dz);
            int64_t hi = (c > 0) ? (int64_t)std::floor((H - zt) / dz) : (int64_t)std::floor((H - zt - reach) / dz);
            while (exists(lo - 1)) --lo;
            while (lo <= hi && !exists(lo)) ++lo;
            while (exists(hi + 1)) ++hi;
            while (hi >= lo && !exists(hi)) --hi;
            ilo[s] = lo;
            cnt[s] = hi >= lo ? hi - lo + 1 : 0;
        }
    }
    T = 64 / group_chunks(G);
    // largest line stride of the windowed sweep's bundles: the lines of one
    // stack per axial layer at a fixed 2D position
    lstride = std::max(1, (int)std::floor(h / dz + 1e-9));
    trk_off.assign(n_stacks + 1, 0);
    chunk_off.assign(n_stacks + 1, 0);
    for (int64_t s = 0; s < n_stacks; ++s) {
        trk_off[s + 1] = trk_off[s] + cnt[s];
        chunk_off[s + 1] = chunk_off[s] + (cnt[s] + T - 1) / T;
    }
    n3d = trk_off[n_stacks];
    n_chunks = chunk_off[n_stacks];

    // ------------------------------------------------ chain-line traversals
    // With vacuum top and bottom faces every z-stack line, continued across
    // the reflective side faces (Eq. 5 along the cycle), runs from one z face
    // to the other, so a sweep can follow it whole.  Each directed cycle is
    // walked from its chain origin (the start of the track C runs forward
    // from chain position 0), where every line of every stack sits at
    // z = (i + 1/2) dz: lines then enter through a z face half an entry
    // spacing away from every segment bound (whole spacings from the origin).
    // A line rises by H over a 2D distance of H / |cot| (its reach), so the
    // lines of a segment [A, B) cross only the units in [A, B + reach).
    n_trav = 0;
    n_chseg = 0;
    ch_first.assign(1, 0);
    ch_code.clear();
    ch_u.clear();
    ch_k.clear();
    ch_nk.clear();
    ch_lc.clear();
    ch_cap = 0;
    if (bc[MOC_FACE_ZMIN] == MOC_BC_VACUUM && bc[MOC_FACE_ZMAX] == MOC_BC_VACUUM) {
        struct Trav {
            std::vector<int64_t> units;
            std::vector<double> spos;
            double lc;
            int az;
        };
        std::vector<Trav> travs;
        for (int64_t t0 = 0; t0 < n2d; ++t0) {
            if (!(sig[t0] == 1 && chain[t0] == 0.0)) continue;
            for (int rev = 0; rev < 2; ++rev) {
                Trav tv;
                tv.az = az[t0];
                const int64_t start = rev ? link[2 * t0 + 1] : 2 * t0;
                double pos = 0.0;
                int64_t u = start;
                do {
                    tv.units.push_back(u);
                    tv.spos.push_back(pos);
                    pos += L[u / 2];
                    u = link[u];
                    if ((int64_t)tv.units.size() > 2 * n2d) return "internal: traversal does not close";
                } while (u != start);
                tv.lc = pos;
                travs.push_back(std::move(tv));
            }
        }
        n_trav = (int64_t)travs.size();
        int64_t covered = 0;
        double total = 0.0, reach_max = 0.0;
        for (const Trav &tv : travs) {
            covered += (int64_t)tv.units.size();
            total += tv.lc;
            for (int n = P / 2; n < P; ++n) reach_max = std::max(reach_max, H / cot[tv.az * P + n]);
        }
        if (covered != 2 * n2d) return "internal: traversals do not cover every unit";
        // segments of about the same length: about 1024 of them to share out
        // the sweep, but from one to four reaches long (a segment's units
        // past its end carry only its last lines, so short segments repeat
        // work: lattice64 ran 4.16 / 4.26 / 4.49 s with segments of 4, 2, 1
        // reaches, lattice8 7.0 / 3.6 / 2.1 ms with 56, 120, 248 segments)
        const double lseg = std::max(reach_max, std::min(4.0 * reach_max, total / 1024.0));
        struct Seg {
            int k, nk;
            double lc;
            std::vector<int> code;
            std::vector<double> u;
        };
        std::vector<Seg> segs;
        for (const Trav &tv : travs) {
            const int nk = (int)std::max(1.0, std::floor(tv.lc / lseg));
            const int m = (int)tv.units.size();
            for (int k = 0; k < nk; ++k) {
                double lo = 1e300, hi = -1e300;
                for (int n = P / 2; n < P; ++n) {
                    const double c = cot[tv.az * P + n];
                    const int64_t kk = std::llround(tv.lc * c / dz);
                    const double sp = tv.lc / (double)kk;
                    const double a0 = (double)((int64_t)k * kk / nk) * sp;
                    const double a1 = (double)((int64_t)(k + 1) * kk / nk) * sp;
                    lo = std::min(lo, a0);
                    hi = std::max(hi, a1 + H / c);
                }
                Seg sg;
                sg.k = k;
                sg.nk = nk;
                sg.lc = tv.lc;
                // from the unit holding lo, in traversal order, until past hi
                int j = (int)(std::upper_bound(tv.spos.begin(), tv.spos.end(), lo) - tv.spos.begin()) - 1;
                j = std::max(j, 0);
                double lap = 0.0;
                for (;;) {
                    const double u = tv.spos[j] + lap;
                    if (u >= hi) break;
                    sg.code.push_back((int)tv.units[j]);
                    sg.u.push_back(u);
                    if (++j == m) {
                        j = 0;
                        lap += tv.lc;
                    }
                }
                segs.push_back(std::move(sg));
            }
        }
        // longest first: workgroups take the next segment as they finish
        std::stable_sort(segs.begin(), segs.end(),
                         [](const Seg &x, const Seg &y) { return x.code.size() > y.code.size(); });
        for (const Seg &sg : segs) {
            ch_code.insert(ch_code.end(), sg.code.begin(), sg.code.end());
            ch_u.insert(ch_u.end(), sg.u.begin(), sg.u.end());
            ch_first.push_back((int)ch_code.size());
            ch_k.push_back(sg.k);
            ch_nk.push_back(sg.nk);
            ch_lc.push_back(sg.lc);
        }
        n_chseg = (int64_t)segs.size();
        for (int64_t s = 0; s < n_stacks; ++s) ch_cap = std::max(ch_cap, cnt[s]);
    }
    return "";
}

moc_plan_info Plan::info() const {
    moc_plan_info o;
    std::memset(&o, 0, sizeof(o));
    o.n_fsr = n_fsr;
    o.n_regions = n_regions;
    o.n_2d_tracks = n2d;
    o.n_2d_segments = (long long)seg_pos.size();
    o.n_stacks = n_stacks;
    o.n_3d_tracks = n3d;
    o.n_chunks = n_chunks;
    o.n_groups = G;
    o.tracks_per_wave = T;
    o.line_stride = lstride;
    o.dz = dz;
    Layout l = make_layout(*this, false);
    o.workspace_bytes = l.total;
    o.psi_bytes = l.psi_bytes;
    o.workspace_bytes_fp64 = make_layout(*this, true).total;
    o.workspace_bytes_chain = n_chseg > 0 ? l.off_psi0 : 0;
    o.n_chain_segments = n_chseg;
    o.n_chain_items = (long long)ch_code.size();
    return o;
}

Layout make_layout(const Plan &p, bool psi64) {
    Layout l;
    l.psi64 = psi64;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    };
    size_t ap = (size_t)p.A2 * p.P;
    l.off_cot = take(ap * 8);
    l.off_secl = take(ap * 8);
    l.off_icot = take(ap * 8);
    l.off_wgt = take(ap * 8);
    l.off_t_len = take(p.n2d * 8);
    l.off_t_first = take((p.n2d + 1) * 4);
    l.off_t_meta = take(p.n2d * 4);
    l.off_t_link = take(2 * p.n2d * 4);
    size_t nseg = p.seg_pos.size();
    l.off_seg_pos = take((nseg + 1) * 8);
    l.off_seg_reg = take((nseg + 1) * 4);
    l.off_seg_st = take((nseg + 1) * (size_t)p.G * 4);
    l.off_reg_mat = take(p.n_regions * 4);
    l.off_zeta = take(p.n_stacks * 8);
    l.off_ilo = take(p.n_stacks * 8);
    l.off_cnt = take(p.n_stacks * 4);
    l.off_trk_off = take((p.n_stacks + 1) * 8);
    l.off_chunk_off = take((p.n_stacks + 1) * 8);
    l.off_sigt32 = take((size_t)p.M * p.G * 4);
    l.off_sigt64 = take((size_t)p.M * p.G * 8);
    l.off_sigs = take((size_t)p.M * p.G * p.G * 8);
    size_t nfg = (size_t)p.n_fsr * p.G;
    l.off_q = take(nfg * 8);
    l.off_qhat32 = take(nfg * 4);
    l.off_qhat64 = take(nfg * 8);
    l.off_acc = take(nfg * 8);
    l.off_phi = take(nfg * 8);
    l.off_vol = take((size_t)p.n_fsr * 8);
    l.off_work = take((size_t)2 * p.n2d * 4);
    l.off_ch_first = take((p.n_chseg + 1) * 4);
    l.off_ch_code = take(p.ch_code.size() * 4 + 4);
    l.off_ch_u = take(p.ch_u.size() * 8 + 8);
    l.off_ch_k = take(p.n_chseg * 4 + 4);
    l.off_ch_nk = take(p.n_chseg * 4 + 4);
    l.off_ch_lc = take(p.n_chseg * 8 + 8);
    l.off_ch_ctr = take(4);
    const size_t slots = p.n_chseg > 0 ? (size_t)std::min<int64_t>(p.n_chseg, kChainSlots) : 0;
    l.off_ch_carry = take(slots * 2 * p.P * (size_t)p.ch_cap * p.G * (psi64 ? 8 : 4));
    l.off_scal = take(128 * 1024);
    l.off_nusf = take((size_t)p.M * p.G * 8);
    l.off_chi = take((size_t)p.M * p.G * 8);
    l.off_fold = take((size_t)p.n_fsr * 8);
    l.n_item_cap = 512;
    l.off_items = take(l.n_item_cap * 8);
    l.off_psi_entry = take(l.n_item_cap * kItemStride * 8);
    l.off_psi_exitb = take(l.n_item_cap * kItemStride * 8);
    l.off_units = take(l.n_item_cap * 4);
    l.off_filt_n = take(l.n_item_cap * 4);
    l.off_filt_i0 = take(l.n_item_cap * 8);
    l.scratch_bytes = off - l.off_items;
    // the two boundary angular-flux buffers last: a chain-only solver (which
    // passes every flux within the sweep) stops short of them
    size_t psi = (size_t)2 * p.n3d * p.G * (psi64 ? 8 : 4);
    l.off_psi0 = take(psi);
    l.off_psi1 = take(psi);
    l.psi_bytes = 2 * ((psi + 255) & ~size_t(255));
    l.total = off;
    return l;
}

}  // namespace moc
