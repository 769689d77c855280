/*
 * FP64 CPU oracle for fixed-source 3D MOC transport (test infrastructure only:
 * it is loaded by the tests, the smoke check and the benchmark's CPU-baseline
 * leg, never by the product path).
 *
 * The oracle is deliberately plain:
 *   - quadrature and 2D cyclic laydown written out from their definitions;
 *   - 2D and 3D reflective links found by matching coordinates and directions;
 *   - 3D tracks taken as the z-stack lines of Eq. 5 (section 2.2) restricted
 *     to the box, and then traced by BRUTE FORCE in 3D against every plane,
 *     circle and sector half-line they cross (no 2D segments, no Eqs. 6-11);
 *   - explicit segment storage, FP64 everywhere, exp via expm1;
 *   - Jacobi source iteration (Eq. 3 per segment, Eq. 4 estimator), with the
 *     boundary flux either lagged one sweep or passed along whole chains of
 *     reflected tracks within the sweep.
 *
 * Readings of points the paper leaves open (quadrature, laydown, chain phase,
 * link scheme, volumes, residual) are listed in the design notes and restated
 * next to the code that implements them.
 */
#include "oracle.h"

#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846
#define MATCH_TOL 1e-9
/* segments shorter than this (cm) are dropped: structural zero-length pieces
 * (a plane crossing that coincides with a surface crossing) carry rounding
 * noise of the chain phase, far below this */
#define MIN_SEG 1e-9
/* a z-stack line is a 3D track only if it runs more than this 2D length
 * inside the box; lines that merely graze a box edge are not tracks */
#define TRACK_EPS 1e-9

/* Planted mistakes for the mutation tests of the pins (0: none).  Each one
 * is a plausible slip in a formula; the pin tests must fail for every one.
 *   1 reduced source without the 1/(4 pi)    4 linearised attenuation (tau)
 *   2 scattering matrix transposed           5 estimator without 4 pi qhat
 *   3 track weight without sin(theta)        6 volumes from one direction
 *   7 fission source without 1/k             8 azimuthal weights from the
 *                                              desired (uncorrected) angles
 *   9 chain sweep that drops the flux at every reflective crossing */
#ifndef ORC_MUTATION
#define ORC_MUTATION 0
#endif
/* 1 - e^{-tau} as the oracle evaluates it (Eq. 3) */
static inline double orc_atten(double tau) {
#if ORC_MUTATION == 4
    return tau;
#else
    return -expm1(-tau);
#endif
}

struct orc_model {
    /* problem */
    int nx, ny, ns, K, G, M, P, A, A2, A4, Rc;
    double pitch, R, H, Wx, Wy, h, dz;
    int bc[6];
    int *cell_mat;
    double *sigt, *sigs;
    long long n_regions, n_fsr;
    int nthreads;
    /* quadrature */
    double *phi, *dphi, *deff, *LC;
    int *nxa, *nya;
    double *mu, *wp, *cot, *wgt;   /* cot, wgt: [A2][P] */
    /* 2D tracks */
    long long n2d, ncyc;
    double *x0, *y0, *x1, *y1, *L, *chain;
    int *az, *f0, *f1, *sig;
    long long *lnk2;               /* [2*n2d] successor directed id */
    /* stacks, Eq. 13 order (azimuth, track within azimuth, polar) */
    long long nstk, n3d;
    double *zeta;
    long long *ilo, *cnt, *off;    /* off: [nstk+1] prefix of cnt */
    /* traced data */
    int traced;
    long long nseg;
    long long *seg_off;            /* [n3d+1] */
    int *seg_fsr;
    double *seg_len;
    long long *succ;               /* [2*n3d] */
    double *vol;
};

/* ------------------------------------------------------------------ */
/* quadrature                                                          */
/* ------------------------------------------------------------------ */

/* Legendre polynomial P_n and its derivative by the three-term recurrence. */
static void legendre(int n, double x, double *pn, double *dpn) {
    double p0 = 1.0, p1 = x;
    if (n == 0) { *pn = 1.0; *dpn = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
    }
    *pn = p1;
    *dpn = n * (x * p1 - p0) / (x * x - 1.0);
}

int orc_gauss_legendre(int n, double *mu, double *w) {
    if (n < 1) return -1;
    /* Newton on P_n for the roots in (0, 1); mirror for the negative half. */
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double x = cos(ORC_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double pn, dpn;
            legendre(n, x, &pn, &dpn);
            double dx = pn / dpn;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        double pn, dpn;
        legendre(n, x, &pn, &dpn);
        double wi = 2.0 / ((1.0 - x * x) * dpn * dpn);
        /* ascending order: largest root last */
        mu[n - 1 - i] = x;
        w[n - 1 - i] = wi;
        mu[i] = -x;
        w[i] = wi;
    }
    if (n % 2 == 1) mu[n / 2] = 0.0;
    return 0;
}

static long long gcdll(long long a, long long b) {
    while (b) { long long t = a % b; a = b; b = t; }
    return a;
}

/* ------------------------------------------------------------------ */
/* coordinate matcher: points on a box face + direction                */
/* ------------------------------------------------------------------ */

typedef struct {
    int face;
    long long qu, qv;
    double u, v;
    double d[3];
    long long id;
} mrec;

#define QSTEP 1e-6

static int mrec_cmp(const void *a, const void *b) {
    const mrec *x = (const mrec *)a, *y = (const mrec *)b;
    if (x->face != y->face) return x->face < y->face ? -1 : 1;
    if (x->qu != y->qu) return x->qu < y->qu ? -1 : 1;
    if (x->qv != y->qv) return x->qv < y->qv ? -1 : 1;
    return 0;
}

/* in-plane coordinates of a point on face f */
static void face_uv(int f, const double *p, double *u, double *v) {
    int axis = f / 2;
    if (axis == 0) { *u = p[1]; *v = p[2]; }
    else if (axis == 1) { *u = p[0]; *v = p[2]; }
    else { *u = p[0]; *v = p[1]; }
}

/* All faces within matching tolerance of p through which d leaves (outward=1)
 * or enters (outward=0); returns the count, faces written to f[]. */
static int faces_of(const struct orc_model *m, const double *p, const double *d, int outward,
                    int dims, int *f) {
    double lo[3] = {0.0, 0.0, 0.0}, hi[3] = {m->Wx, m->Wy, m->H};
    int n = 0;
    for (int axis = 0; axis < dims; ++axis) {
        for (int side = 0; side < 2; ++side) {
            double dist = fabs(p[axis] - (side ? hi[axis] : lo[axis]));
            double dn = (side ? 1.0 : -1.0) * d[axis];
            if ((outward ? (dn > 0) : (dn < 0)) && dist < MATCH_TOL) f[n++] = 2 * axis + side;
        }
    }
    return n;
}

static void mrec_fill(mrec *r, int face, const double *p, const double *d, long long id) {
    r->face = face;
    face_uv(face, p, &r->u, &r->v);
    r->qu = (long long)floor(r->u / QSTEP);
    r->qv = (long long)floor(r->v / QSTEP);
    r->d[0] = d[0]; r->d[1] = d[1]; r->d[2] = d[2];
    r->id = id;
}

/* returns matching id, -1 when none, -2 when ambiguous */
static long long mrec_find(const mrec *tab, long long n, int face, const double *p, const double *d) {
    double u, v;
    face_uv(face, p, &u, &v);
    long long qu = (long long)floor(u / QSTEP), qv = (long long)floor(v / QSTEP);
    long long found = -1;
    for (int du = -1; du <= 1; ++du) {
        for (int dv = -1; dv <= 1; ++dv) {
            mrec key;
            key.face = face; key.qu = qu + du; key.qv = qv + dv;
            long long lo = 0, hi = n;
            while (lo < hi) {
                long long mid = (lo + hi) / 2;
                if (mrec_cmp(&tab[mid], &key) < 0) lo = mid + 1; else hi = mid;
            }
            for (long long i = lo; i < n && mrec_cmp(&tab[i], &key) == 0; ++i) {
                const mrec *r = &tab[i];
                if (fabs(r->u - u) > MATCH_TOL || fabs(r->v - v) > MATCH_TOL) continue;
                double dot = r->d[0] * d[0] + r->d[1] * d[1] + r->d[2] * d[2];
                if (dot < 1.0 - 1e-10) continue;
                if (found >= 0 && found != r->id) return -2;
                found = r->id;
            }
        }
    }
    return found;
}

/* ------------------------------------------------------------------ */
/* geometry: FSR of a point                                             */
/* ------------------------------------------------------------------ */

static long long fsr_at(const struct orc_model *m, double x, double y, double z, int *mat_out) {
    int cx = (int)floor(x / m->pitch), cy = (int)floor(y / m->pitch);
    if (cx < 0) cx = 0;
    if (cx >= m->nx) cx = m->nx - 1;
    if (cy < 0) cy = 0;
    if (cy >= m->ny) cy = m->ny - 1;
    int k = (int)floor(z / m->h);
    if (k < 0) k = 0;
    if (k >= m->K) k = m->K - 1;
    double dx = x - (cx + 0.5) * m->pitch, dy = y - (cy + 0.5) * m->pitch;
    int inside = 0;
    if (m->R > 0) inside = (dx * dx + dy * dy) < m->R * m->R;
    int s = 0;
    if (m->ns > 1) {
        double ang = atan2(dy, dx);
        if (ang < 0) ang += 2.0 * ORC_PI;
        /* a point within 1e-9 of a sector line belongs to the sector that
         * starts at that line (tracks that run along a sector line) */
        s = ((int)floor(ang / (2.0 * ORC_PI / m->ns) + 1e-9)) % m->ns;
        if (s < 0) s = 0;
    }
    int local = (m->R > 0) ? 2 * s + (inside ? 0 : 1) : s;
    int cell = cy * m->nx + cx;
    if (mat_out) *mat_out = m->cell_mat[2 * cell + (inside ? 0 : 1)];
    long long r = (long long)cell * m->Rc + local;
    return r * m->K + k;
}

static int dcmp(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) ? -1 : (x > y) ? 1 : 0;
}

/* Brute-force 3D tracing of the straight segment p0 -> p1.  Every crossing of
 * a cell plane, axial plane, inclusion circle or sector half-line inside the
 * segment is collected, the crossings are sorted, each interval is assigned
 * the FSR containing its midpoint, intervals shorter than MIN_SEG are dropped
 * and consecutive intervals of the same FSR are merged.  Writes up to cap
 * segments and returns the count (which may exceed cap). */
static long long trace3d(const struct orc_model *m, const double *p0, const double *p1,
                         int *fsr, double *len, long long cap) {
    double D[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
    double T = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
    if (!(T > 0)) return 0;
    double d[3] = {D[0] / T, D[1] / T, D[2] / T};
    long long ncap = 2 * (m->nx + m->ny + m->K) + 64;
    double *ts = (double *)malloc(sizeof(double) * ncap);
    long long nt = 0;
#define PUSH(val) do { if (nt >= ncap) { ncap *= 2; ts = (double *)realloc(ts, sizeof(double) * ncap); } ts[nt++] = (val); } while (0)
    /* radial cell planes */
    for (int k = 1; k < m->nx; ++k) {
        if (d[0] != 0.0) { double t = (k * m->pitch - p0[0]) / d[0]; if (t > 0 && t < T) PUSH(t); }
    }
    for (int k = 1; k < m->ny; ++k) {
        if (d[1] != 0.0) { double t = (k * m->pitch - p0[1]) / d[1]; if (t > 0 && t < T) PUSH(t); }
    }
    long long n_cellcross = nt;
    /* axial planes */
    for (int k = 1; k < m->K; ++k) {
        if (d[2] != 0.0) { double t = (k * m->h - p0[2]) / d[2]; if (t > 0 && t < T) PUSH(t); }
    }
    /* inclusion circles and sector half-lines of every cell the track visits */
    if (m->R > 0 || m->ns > 1) {
        double *cc = (double *)malloc(sizeof(double) * (n_cellcross + 2));
        cc[0] = 0.0;
        memcpy(cc + 1, ts, sizeof(double) * n_cellcross);
        cc[n_cellcross + 1] = T;
        qsort(cc + 1, n_cellcross, sizeof(double), dcmp);
        double dxy2 = d[0] * d[0] + d[1] * d[1];
        for (long long iv = 0; iv <= n_cellcross; ++iv) {
            double ta = cc[iv], tb = cc[iv + 1];
            double tm = 0.5 * (ta + tb);
            double xm = p0[0] + tm * d[0], ym = p0[1] + tm * d[1];
            int cx = (int)floor(xm / m->pitch), cy = (int)floor(ym / m->pitch);
            if (cx < 0) cx = 0;
            if (cx >= m->nx) cx = m->nx - 1;
            if (cy < 0) cy = 0;
            if (cy >= m->ny) cy = m->ny - 1;
            double cxc = (cx + 0.5) * m->pitch, cyc = (cy + 0.5) * m->pitch;
            double wx = cxc - p0[0], wy = cyc - p0[1];
            if (m->R > 0 && dxy2 > 0) {
                /* |p0 + t d - c|^2 = R^2 in the xy projection */
                double a = dxy2;
                double b = -2.0 * (wx * d[0] + wy * d[1]);
                double c = wx * wx + wy * wy - m->R * m->R;
                double disc = b * b - 4 * a * c;
                if (disc > 0) {
                    double sq = sqrt(disc);
                    double r1 = (-b - sq) / (2 * a), r2 = (-b + sq) / (2 * a);
                    if (r1 > ta && r1 < tb) PUSH(r1);
                    if (r2 > ta && r2 < tb) PUSH(r2);
                }
            }
            if (m->ns > 1 && dxy2 > 0) {
                /* with an even sector count the half-lines at angle a and
                 * a + pi are both sector boundaries: intersect the full lines
                 * through the cell centre (a track through the centre then
                 * splits there whatever the rounding) */
                for (int s = 0; s < m->ns / 2; ++s) {
                    double al = 2.0 * ORC_PI * s / m->ns;
                    double ex = cos(al), ey = sin(al);
                    double dxe = d[0] * ey - d[1] * ex;     /* d x e */
                    if (dxe == 0.0) continue;
                    double t = (wx * ey - wy * ex) / dxe;   /* (w x e)/(d x e) */
                    if (t > ta && t < tb) PUSH(t);
                }
            }
        }
        free(cc);
    }
#undef PUSH
    qsort(ts, nt, sizeof(double), dcmp);
    long long nseg = 0;
    long long last_fsr = -1;
    double prev = 0.0;
    for (long long i = 0; i <= nt; ++i) {
        double t1 = (i < nt) ? ts[i] : T;
        double l = t1 - prev;
        if (l >= MIN_SEG) {
            double tm = 0.5 * (prev + t1);
            long long f = fsr_at(m, p0[0] + tm * d[0], p0[1] + tm * d[1], p0[2] + tm * d[2], NULL);
            if (f == last_fsr && nseg > 0) {
                if (nseg - 1 < cap) len[nseg - 1] += l;
            } else {
                if (nseg < cap) { fsr[nseg] = (int)f; len[nseg] = l; }
                ++nseg;
                last_fsr = f;
            }
        }
        prev = t1;
    }
    free(ts);
    return nseg;
}

/* ------------------------------------------------------------------ */
/* laydown                                                              */
/* ------------------------------------------------------------------ */

static int build_quadrature(struct orc_model *m, const orc_problem *p) {
    int A2 = m->A2, A4 = m->A4, P = m->P;
    m->phi = calloc(A2, sizeof(double));
    m->dphi = calloc(A2, sizeof(double));
    m->deff = calloc(A2, sizeof(double));
    m->LC = calloc(A2, sizeof(double));
    m->nxa = calloc(A2, sizeof(int));
    m->nya = calloc(A2, sizeof(int));
    m->mu = calloc(P, sizeof(double));
    m->wp = calloc(P, sizeof(double));
    m->cot = calloc((size_t)A2 * P, sizeof(double));
    m->wgt = calloc((size_t)A2 * P, sizeof(double));
    /* azimuths of the first quadrant: desired angle, track counts per side,
     * corrected angle that makes tracks cyclic, corrected spacing */
    for (int a = 0; a < A4; ++a) {
        double phid = 2.0 * ORC_PI / m->A * (a + 0.5);
        m->nxa[a] = (int)ceil(m->Wx / p->radial_spacing * fabs(sin(phid)));
        m->nya[a] = (int)ceil(m->Wy / p->radial_spacing * fabs(cos(phid)));
        m->phi[a] = atan((m->Wy * m->nxa[a]) / (m->Wx * m->nya[a]));
        m->deff[a] = (m->Wx / m->nxa[a]) * sin(m->phi[a]);
    }
    /* second quadrant mirrors the first */
    for (int a = A4; a < A2; ++a) {
        int am = A2 - 1 - a;
        m->nxa[a] = m->nxa[am];
        m->nya[a] = m->nya[am];
        m->phi[a] = ORC_PI - m->phi[am];
        m->deff[a] = m->deff[am];
    }
    /* azimuthal weights: half the gap between neighbouring corrected angles */
    for (int a = 0; a < A4; ++a) {
        double prev = (a == 0) ? -m->phi[0] : m->phi[a - 1];
        double next = (a == A4 - 1) ? ORC_PI - m->phi[A4 - 1] : m->phi[a + 1];
#if ORC_MUTATION == 8
        /* the same rule on the desired angles: every gap is 2 pi / A */
        prev = 2.0 * ORC_PI / m->A * (a - 0.5);
        next = 2.0 * ORC_PI / m->A * (a + 1.5);
#endif
        m->dphi[a] = 0.5 * (next - prev);
        m->dphi[A2 - 1 - a] = m->dphi[a];
    }
    for (int a = 0; a < A2; ++a) {
        double g = (double)gcdll(m->nxa[a], m->nya[a]);
        double lx = 2.0 * m->Wx * m->nya[a] / g, ly = 2.0 * m->Wy * m->nxa[a] / g;
        m->LC[a] = sqrt(lx * lx + ly * ly);
    }
    orc_gauss_legendre(P, m->mu, m->wp);
    /* polar angles: corrected per azimuth so the 3D lines close after one
     * cycle (an integer number of axial spacings per cycle length) */
    for (int a = 0; a < A2; ++a) {
        for (int n = P / 2; n < P; ++n) {
            double mu = m->mu[n];
            double cot0 = mu / sqrt(1.0 - mu * mu);
            double kk = floor(m->LC[a] * cot0 / m->dz + 0.5);
            if (kk < 1) kk = 1;
            double c = kk * m->dz / m->LC[a];
            m->cot[a * P + n] = c;
            m->cot[a * P + (P - 1 - n)] = -c;
        }
        for (int n = 0; n < P; ++n) {
            double c = m->cot[a * P + n];
            double sint = 1.0 / sqrt(1.0 + c * c);
            double wpol = m->wp[n >= P / 2 ? n : P - 1 - n];
            /* solid-angle weight x perpendicular area per 3D track */
#if ORC_MUTATION == 3
            sint = 1.0;
#endif
            m->wgt[a * P + n] = m->dphi[a] * wpol * m->deff[a] * m->dz * sint;
        }
    }
    return 0;
}

static int build_tracks2d(struct orc_model *m) {
    long long n = 0;
    for (int a = 0; a < m->A2; ++a) n += m->nxa[a] + m->nya[a];
    m->n2d = n;
    m->x0 = calloc(n, sizeof(double)); m->y0 = calloc(n, sizeof(double));
    m->x1 = calloc(n, sizeof(double)); m->y1 = calloc(n, sizeof(double));
    m->L = calloc(n, sizeof(double)); m->chain = calloc(n, sizeof(double));
    m->az = calloc(n, sizeof(int)); m->f0 = calloc(n, sizeof(int));
    m->f1 = calloc(n, sizeof(int)); m->sig = calloc(n, sizeof(int));
    m->lnk2 = calloc(2 * n, sizeof(long long));
    long long t = 0;
    for (int a = 0; a < m->A2; ++a) {
        double ux = cos(m->phi[a]), uy = sin(m->phi[a]);
        int right = (a >= m->A4);
        for (int i = 0; i < m->nxa[a] + m->nya[a]; ++i, ++t) {
            double xs, ys;
            if (i < m->nxa[a]) { xs = (i + 0.5) * m->Wx / m->nxa[a]; ys = 0.0; m->f0[t] = 2; }
            else {
                int j = i - m->nxa[a];
                xs = right ? m->Wx : 0.0;
                ys = (j + 0.5) * m->Wy / m->nya[a];
                m->f0[t] = right ? 1 : 0;
            }
            double tx = (ux > 0) ? (m->Wx - xs) / ux : (0.0 - xs) / ux;
            double ty = (m->Wy - ys) / uy;
            double L, xe, ye;
            if (ty < tx) { L = ty; xe = xs + L * ux; ye = m->Wy; m->f1[t] = 3; }
            else { L = tx; xe = (ux > 0) ? m->Wx : 0.0; ye = ys + L * uy; m->f1[t] = (ux > 0) ? 1 : 0; }
            m->x0[t] = xs; m->y0[t] = ys; m->x1[t] = xe; m->y1[t] = ye; m->L[t] = L; m->az[t] = a;
        }
    }
    /* 2D reflective links by matching exit point + reflected direction against
     * the start points of all directed 2D tracks */
    mrec *tab = calloc(4 * n, sizeof(mrec));
    long long ntab = 0;
    for (long long tt = 0; tt < n; ++tt) {
        double ux = cos(m->phi[m->az[tt]]), uy = sin(m->phi[m->az[tt]]);
        double pf[3] = {m->x0[tt], m->y0[tt], 0}, df[3] = {ux, uy, 0};
        double pb[3] = {m->x1[tt], m->y1[tt], 0}, db[3] = {-ux, -uy, 0};
        int fl[6];
        int nf = faces_of(m, pf, df, 0, 2, fl);
        if (nf < 1) { free(tab); return -10; }
        for (int i = 0; i < nf; ++i) mrec_fill(&tab[ntab++], fl[i], pf, df, 2 * tt);
        nf = faces_of(m, pb, db, 0, 2, fl);
        if (nf < 1) { free(tab); return -10; }
        for (int i = 0; i < nf; ++i) mrec_fill(&tab[ntab++], fl[i], pb, db, 2 * tt + 1);
    }
    qsort(tab, ntab, sizeof(mrec), mrec_cmp);
    for (long long tt = 0; tt < n; ++tt) {
        double ux = cos(m->phi[m->az[tt]]), uy = sin(m->phi[m->az[tt]]);
        for (int dir = 0; dir < 2; ++dir) {
            double pe[3] = {dir ? m->x0[tt] : m->x1[tt], dir ? m->y0[tt] : m->y1[tt], 0};
            double de[3] = {dir ? -ux : ux, dir ? -uy : uy, 0};
            int fl[6];
            int nf = faces_of(m, pe, de, 1, 2, fl);
            if (nf < 1) { free(tab); return -11; }
            for (int i = 0; i < nf; ++i) de[fl[i] / 2] = -de[fl[i] / 2];
            long long s = mrec_find(tab, ntab, fl[0], pe, de);
            if (s < 0) { free(tab); return -12; }
            m->lnk2[2 * tt + dir] = s;
        }
    }
    free(tab);
    /* cycles and chain coordinates: for each pair of mutually reversed
     * directed cycles, C is the one that runs the lowest-id track forward and
     * the chain coordinate is measured along C from that track's start */
    char *seen = calloc(n, 1);
    m->ncyc = 0;
    for (long long t0 = 0; t0 < n; ++t0) {
        if (seen[t0]) continue;
        long long cur = 2 * t0;
        double pos = 0.0;
        long long steps = 0;
        do {
            long long tt = cur / 2;
            int dir = (int)(cur % 2);
            if (seen[tt]) { free(seen); return -13; }   /* C would equal its reverse */
            seen[tt] = 1;
            if (dir == 0) { m->chain[tt] = pos; m->sig[tt] = 1; }
            else { m->chain[tt] = pos + m->L[tt]; m->sig[tt] = -1; }
            pos += m->L[tt];
            cur = m->lnk2[cur];
            if (++steps > 2 * n) { free(seen); return -14; }
        } while (cur != 2 * t0);
        if (fabs(pos - m->LC[m->az[t0]]) > 1e-9 * m->LC[m->az[t0]]) { free(seen); return -15; }
        m->ncyc += 2;
    }
    free(seen);
    return 0;
}

/* clip line z = base + c*l to 0 <= l <= L, 0 <= z <= H */
static void clip_line(double base, double c, double L, double H, double *ls, double *le) {
    double a, b;
    if (c > 0) { a = -base / c; b = (H - base) / c; }
    else { a = (H - base) / c; b = -base / c; }
    *ls = a > 0 ? a : 0.0;
    *le = b < L ? b : L;
}

static int build_stacks(struct orc_model *m) {
    m->nstk = m->n2d * m->P;
    m->zeta = calloc(m->nstk, sizeof(double));
    m->ilo = calloc(m->nstk, sizeof(long long));
    m->cnt = calloc(m->nstk, sizeof(long long));
    m->off = calloc(m->nstk + 1, sizeof(long long));
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) num_threads(m->nthreads) reduction(|:bad)
    for (long long t = 0; t < m->n2d; ++t) {
        for (int n = 0; n < m->P; ++n) {
            long long s = t * m->P + n;
            double c = m->cot[m->az[t] * m->P + n];
            /* Eq. 5 with the chain phase: z0 = dz/2 + sigma * cot * a (mod dz) */
            double zeta = fmod(0.5 * m->dz + m->sig[t] * c * m->chain[t], m->dz);
            if (zeta < 0) zeta += m->dz;
            if (zeta >= m->dz) zeta -= m->dz;
            m->zeta[s] = zeta;
            /* enumerate candidate lines generously and keep those with a
             * positive-length intersection with the (l, z) rectangle */
            double reach = fabs(c) * m->L[t];
            long long i0 = (long long)floor((-reach - zeta) / m->dz) - 2;
            long long i1 = (long long)ceil((m->H + reach - zeta) / m->dz) + 2;
            long long first = 0, count = 0;
            for (long long i = i0; i <= i1; ++i) {
                double ls, le;
                clip_line(zeta + i * m->dz, c, m->L[t], m->H, &ls, &le);
                if (le - ls > TRACK_EPS) {
                    if (count == 0) first = i;
                    else if (i != first + count) bad = 1;   /* not contiguous */
                    ++count;
                }
            }
            m->ilo[s] = first;
            m->cnt[s] = count;
        }
    }
    if (bad) return -20;
    m->off[0] = 0;
    for (long long s = 0; s < m->nstk; ++s) m->off[s + 1] = m->off[s] + m->cnt[s];
    m->n3d = m->off[m->nstk];
    return 0;
}

static long long stack_of(const struct orc_model *m, long long track) {
    long long lo = 0, hi = m->nstk;   /* largest s with off[s] <= track */
    while (hi - lo > 1) {
        long long mid = (lo + hi) / 2;
        if (m->off[mid] <= track) lo = mid; else hi = mid;
    }
    return lo;
}

/* endpoints of stored 3D track, and its direction (unit) */
static void track_endpoints(const struct orc_model *m, long long track, double *p0, double *p1,
                            double *dir, double *ls_out, double *le_out) {
    long long s = stack_of(m, track);
    long long t = s / m->P;
    int n = (int)(s % m->P);
    int a = m->az[t];
    double c = m->cot[a * m->P + n];
    double base = m->zeta[s] + (double)(m->ilo[s] + (track - m->off[s])) * m->dz;
    double ls, le;
    clip_line(base, c, m->L[t], m->H, &ls, &le);
    double ux = cos(m->phi[a]), uy = sin(m->phi[a]);
    p0[0] = m->x0[t] + ls * ux; p0[1] = m->y0[t] + ls * uy; p0[2] = base + c * ls;
    p1[0] = m->x0[t] + le * ux; p1[1] = m->y0[t] + le * uy; p1[2] = base + c * le;
    /* snap end points exactly onto the box face they lie on */
    if (ls == 0.0) { p0[0] = m->x0[t]; p0[1] = m->y0[t]; }
    else p0[2] = (c > 0) ? 0.0 : m->H;
    if (le == m->L[t]) { p1[0] = m->x1[t]; p1[1] = m->y1[t]; }
    else p1[2] = (c > 0) ? m->H : 0.0;
    double s3 = sqrt(1.0 + c * c);
    dir[0] = ux / s3; dir[1] = uy / s3; dir[2] = c / s3;
    if (ls_out) *ls_out = ls;
    if (le_out) *le_out = le;
}

double orc_track_weight(const orc_model *m, long long track) {
    long long s = stack_of(m, track);
    long long t = s / m->P;
    return m->wgt[m->az[t] * m->P + (int)(s % m->P)];
}

static int build_traced(struct orc_model *m) {
    long long n3 = m->n3d;
    m->seg_off = calloc(n3 + 1, sizeof(long long));
    long long *nseg = calloc(n3, sizeof(long long));
    /* pass 1: count segments per track */
#pragma omp parallel num_threads(m->nthreads)
    {
        long long cap = 4096;
        int *f = malloc(sizeof(int) * cap);
        double *l = malloc(sizeof(double) * cap);
#pragma omp for schedule(dynamic, 256)
        for (long long tr = 0; tr < n3; ++tr) {
            double p0[3], p1[3], d[3];
            track_endpoints(m, tr, p0, p1, d, NULL, NULL);
            long long k = trace3d(m, p0, p1, f, l, 0);
            nseg[tr] = k;
        }
        free(f); free(l);
    }
    m->seg_off[0] = 0;
    for (long long tr = 0; tr < n3; ++tr) m->seg_off[tr + 1] = m->seg_off[tr] + nseg[tr];
    free(nseg);
    m->nseg = m->seg_off[n3];
    m->seg_fsr = malloc(sizeof(int) * (m->nseg + 1));
    m->seg_len = malloc(sizeof(double) * (m->nseg + 1));
    /* pass 2: store */
#pragma omp parallel for schedule(dynamic, 256) num_threads(m->nthreads)
    for (long long tr = 0; tr < n3; ++tr) {
        double p0[3], p1[3], d[3];
        track_endpoints(m, tr, p0, p1, d, NULL, NULL);
        long long b = m->seg_off[tr];
        trace3d(m, p0, p1, m->seg_fsr + b, m->seg_len + b, m->seg_off[tr + 1] - b);
    }
    /* 3D links by coordinate + direction matching over all directed starts */
    /* every directed start is registered under each face it lies on, so a
     * start on a box edge is found whichever of its faces is queried */
    mrec *tab = malloc(sizeof(mrec) * 6 * n3);
    int *nrec = calloc(2 * n3, sizeof(int));
    int bad = 0;
#pragma omp parallel for schedule(static) num_threads(m->nthreads) reduction(|:bad)
    for (long long tr = 0; tr < n3; ++tr) {
        double p0[3], p1[3], d[3], db[3];
        track_endpoints(m, tr, p0, p1, d, NULL, NULL);
        db[0] = -d[0]; db[1] = -d[1]; db[2] = -d[2];
        int fl[6];
        int nf = faces_of(m, p0, d, 0, 3, fl);
        if (nf < 1 || nf > 3) bad = 1;
        for (int i = 0; i < nf && i < 3; ++i) mrec_fill(&tab[6 * tr + i], fl[i], p0, d, 2 * tr);
        nrec[2 * tr] = nf < 3 ? nf : 3;
        nf = faces_of(m, p1, db, 0, 3, fl);
        if (nf < 1 || nf > 3) bad = 1;
        for (int i = 0; i < nf && i < 3; ++i) mrec_fill(&tab[6 * tr + 3 + i], fl[i], p1, db, 2 * tr + 1);
        nrec[2 * tr + 1] = nf < 3 ? nf : 3;
    }
    if (bad) { free(tab); free(nrec); return -30; }
    long long ntab = 0;
    for (long long k = 0; k < 2 * n3; ++k) {
        for (int i = 0; i < nrec[k]; ++i) tab[ntab++] = tab[3 * k + i];
    }
    free(nrec);
    qsort(tab, ntab, sizeof(mrec), mrec_cmp);
    m->succ = malloc(sizeof(long long) * 2 * n3);
#pragma omp parallel for schedule(static) num_threads(m->nthreads) reduction(|:bad)
    for (long long tr = 0; tr < n3; ++tr) {
        double p0[3], p1[3], d[3];
        track_endpoints(m, tr, p0, p1, d, NULL, NULL);
        for (int dir = 0; dir < 2; ++dir) {
            double *pe = dir ? p0 : p1;
            double de[3] = {dir ? -d[0] : d[0], dir ? -d[1] : d[1], dir ? -d[2] : d[2]};
            /* leave through every face the exit point lies on (a box edge is
             * two faces): vacuum if any of them is vacuum, else the specular
             * reflection across all of them */
            int fl[6];
            int nf = faces_of(m, pe, de, 1, 3, fl);
            if (nf < 1) { bad = 1; continue; }
            int vac = 0;
            for (int i = 0; i < nf; ++i) vac |= (m->bc[fl[i]] == 0);
            if (vac) { m->succ[2 * tr + dir] = -1; continue; }
            for (int i = 0; i < nf; ++i) de[fl[i] / 2] = -de[fl[i] / 2];
            long long s = mrec_find(tab, ntab, fl[0], pe, de);
            if (s < 0) { bad = 1; s = -1; }
            m->succ[2 * tr + dir] = s;
        }
    }
    free(tab);
    if (bad) return -31;
    /* track-estimated volumes: V = (1/4pi) sum over directed segments W l */
    m->vol = calloc(m->n_fsr, sizeof(double));
    for (long long tr = 0; tr < n3; ++tr) {
        double w = orc_track_weight(m, tr);
        for (long long k = m->seg_off[tr]; k < m->seg_off[tr + 1]; ++k)
            m->vol[m->seg_fsr[k]] += (ORC_MUTATION == 6 ? 1.0 : 2.0) * w * m->seg_len[k] / (4.0 * ORC_PI);
    }
    m->traced = 1;
    return 0;
}

int orc_build(const orc_problem *p, int trace, int n_threads, orc_model **out) {
    *out = NULL;
    if (p->n_azim < 4 || p->n_azim % 4 != 0) return -1;
    if (p->n_polar < 2 || p->n_polar % 2 != 0) return -1;
    if (!(p->radial_spacing > 0) || !(p->axial_spacing > 0)) return -1;
    if (p->nx < 1 || p->ny < 1 || !(p->pitch > 0) || p->n_layers < 1 || !(p->height > 0)) return -1;
    if (p->radius < 0 || p->radius >= 0.5 * p->pitch) return -1;
    if (p->n_sectors < 1) return -1;
    if (p->n_groups < 1 || p->n_materials < 1) return -1;
    struct orc_model *m = calloc(1, sizeof(struct orc_model));
    m->nx = p->nx; m->ny = p->ny; m->ns = p->n_sectors; m->K = p->n_layers;
    m->G = p->n_groups; m->M = p->n_materials; m->P = p->n_polar; m->A = p->n_azim;
    m->A2 = m->A / 2; m->A4 = m->A / 4;
    m->pitch = p->pitch; m->R = p->radius; m->H = p->height;
    m->Wx = p->nx * p->pitch; m->Wy = p->ny * p->pitch; m->h = p->height / p->n_layers;
    m->dz = p->height / ceil(p->height / p->axial_spacing);
    memcpy(m->bc, p->bc, sizeof(m->bc));
    m->Rc = (p->radius > 0 ? 2 : 1) * p->n_sectors;
    m->n_regions = (long long)p->nx * p->ny * m->Rc;
    m->n_fsr = m->n_regions * m->K;
    m->nthreads = n_threads > 0 ? n_threads : omp_get_max_threads();
    m->cell_mat = malloc(sizeof(int) * 2 * p->nx * p->ny);
    memcpy(m->cell_mat, p->cell_material, sizeof(int) * 2 * p->nx * p->ny);
    m->sigt = malloc(sizeof(double) * m->M * m->G);
    memcpy(m->sigt, p->sigma_t, sizeof(double) * m->M * m->G);
    m->sigs = malloc(sizeof(double) * m->M * m->G * m->G);
    memcpy(m->sigs, p->sigma_s, sizeof(double) * m->M * m->G * m->G);
    int rc = build_quadrature(m, p);
    if (!rc) rc = build_tracks2d(m);
    if (!rc) rc = build_stacks(m);
    if (!rc && trace) rc = build_traced(m);
    if (rc) { orc_free(m); return rc; }
    *out = m;
    return 0;
}

void orc_free(orc_model *m) {
    if (!m) return;
    void *ptrs[] = {m->cell_mat, m->sigt, m->sigs, m->phi, m->dphi, m->deff, m->LC, m->nxa, m->nya,
                    m->mu, m->wp, m->cot, m->wgt, m->x0, m->y0, m->x1, m->y1, m->L, m->chain,
                    m->az, m->f0, m->f1, m->sig, m->lnk2, m->zeta, m->ilo, m->cnt, m->off,
                    m->seg_off, m->seg_fsr, m->seg_len, m->succ, m->vol};
    for (size_t i = 0; i < sizeof(ptrs) / sizeof(ptrs[0]); ++i) free(ptrs[i]);
    free(m);
}

void orc_get_info(const orc_model *m, orc_info *o) {
    o->n_fsr = m->n_fsr; o->n_regions = m->n_regions; o->n_2d_tracks = m->n2d;
    o->n_3d_tracks = m->n3d; o->n_segments = m->traced ? m->nseg : -1;
    o->n_cycles = m->ncyc; o->dz = m->dz; o->traced = m->traced;
}

void orc_get_quadrature(const orc_model *m, double *phi_eff, double *dphi, double *spacing_eff,
                        int *nx_a, int *ny_a, double *mu, double *wpol, double *cot_eff,
                        double *weight) {
    for (int a = 0; a < m->A2; ++a) {
        phi_eff[a] = m->phi[a]; dphi[a] = m->dphi[a]; spacing_eff[a] = m->deff[a];
        nx_a[a] = m->nxa[a]; ny_a[a] = m->nya[a];
    }
    for (int n = 0; n < m->P; ++n) { mu[n] = m->mu[n]; wpol[n] = m->wp[n]; }
    for (int i = 0; i < m->A2 * m->P; ++i) { cot_eff[i] = m->cot[i]; weight[i] = m->wgt[i]; }
}

void orc_get_tracks2d(const orc_model *m, double *xy, double *len, int *azim, int *faces,
                      long long *link2d, double *chain, int *sigma) {
    for (long long t = 0; t < m->n2d; ++t) {
        xy[4 * t] = m->x0[t]; xy[4 * t + 1] = m->y0[t]; xy[4 * t + 2] = m->x1[t]; xy[4 * t + 3] = m->y1[t];
        len[t] = m->L[t]; azim[t] = m->az[t]; faces[2 * t] = m->f0[t]; faces[2 * t + 1] = m->f1[t];
        link2d[2 * t] = m->lnk2[2 * t]; link2d[2 * t + 1] = m->lnk2[2 * t + 1];
        chain[t] = m->chain[t]; sigma[t] = m->sig[t];
    }
}

void orc_get_stacks(const orc_model *m, double *zeta, long long *i_lo, long long *count) {
    for (long long s = 0; s < m->nstk; ++s) { zeta[s] = m->zeta[s]; i_lo[s] = m->ilo[s]; count[s] = m->cnt[s]; }
}

long long orc_trace_track(const orc_model *m, long long track, int *fsr, double *len, long long cap) {
    if (track < 0 || track >= m->n3d) return -1;
    double p0[3], p1[3], d[3];
    track_endpoints(m, track, p0, p1, d, NULL, NULL);
    return trace3d(m, p0, p1, fsr, len, cap);
}

int orc_track_info(const orc_model *m, long long track, double *p01, long long *succ) {
    if (track < 0 || track >= m->n3d) return -1;
    double d[3];
    track_endpoints(m, track, p01, p01 + 3, d, NULL, NULL);
    if (succ) {
        if (!m->traced) return -2;
        succ[0] = m->succ[2 * track]; succ[1] = m->succ[2 * track + 1];
    }
    return 0;
}

int orc_sample_path_length(const orc_model *m, long long n_items, const long long *track,
                           double *wl, long long *n_seg_out) {
    long long total = 0, cap = 1 << 16;
    int bad = 0;
    int *f = malloc(sizeof(int) * cap);
    double *l = malloc(sizeof(double) * cap);
    for (long long it = 0; it < n_items && !bad; ++it) {
        long long tr = track[it];
        if (tr < 0 || tr >= m->n3d) { bad = 1; break; }
        double p0[3], p1[3], d[3];
        track_endpoints(m, tr, p0, p1, d, NULL, NULL);
        long long ns = trace3d(m, p0, p1, f, l, cap);
        if (ns > cap) { bad = 1; break; }
        total += ns;
        double w = orc_track_weight(m, tr);
        /* the volume estimator of the track-length flux estimate, one
         * direction of the listed tracks: sum of W l per FSR */
        for (long long k = 0; k < ns; ++k) wl[f[k]] += w * l[k];
    }
    free(f); free(l);
    if (n_seg_out) *n_seg_out = total;
    return bad ? -1 : 0;
}

int orc_entry_vacuum(const orc_model *m, long long track, int dir) {
    if (track < 0 || track >= m->n3d || (dir != 0 && dir != 1)) return -1;
    double p0[3], p1[3], d[3];
    track_endpoints(m, track, p0, p1, d, NULL, NULL);
    /* the directed track enters at p0 moving along d (forward) or at p1
     * moving along -d (backward); through a box edge it enters through both
     * faces, and a vacuum face among them gives no incoming flux */
    const double *pe = dir ? p1 : p0;
    double de[3] = {dir ? -d[0] : d[0], dir ? -d[1] : d[1], dir ? -d[2] : d[2]};
    int fl[6];
    int nf = faces_of(m, pe, de, 0, 3, fl);
    if (nf < 1) return -2;
    for (int i = 0; i < nf; ++i)
        if (m->bc[fl[i]] == 0) return 1;
    return 0;
}

int orc_segment_counts(const orc_model *m, long long *counts) {
    if (!m->traced) return -2;
    for (long long tr = 0; tr < m->n3d; ++tr) counts[tr] = m->seg_off[tr + 1] - m->seg_off[tr];
    return 0;
}

int orc_volumes(const orc_model *m, double *vol) {
    if (!m->traced) return -2;
    memcpy(vol, m->vol, sizeof(double) * m->n_fsr);
    return 0;
}

/* ------------------------------------------------------------------ */
/* source iteration                                                     */
/* ------------------------------------------------------------------ */

static int fsr_material(const struct orc_model *m, long long j) {
    long long r = j / m->K;
    int cell = (int)(r / m->Rc), local = (int)(r % m->Rc);
    int inside = (m->R > 0) ? ((local % 2) == 0) : 0;
    return m->cell_mat[2 * cell + (inside ? 0 : 1)];
}

/* Eq. 3 along one directed 3D track: psi (the incoming flux on entry) leaves
 * as the outgoing flux; acc += w * delta psi of every segment (Eq. 4). */
static void track_sweep(const struct orc_model *m, long long dt, const double *qhat,
                        const int *mat, double w, double *psi, double *acc) {
    const int G = m->G;
    long long tr = dt / 2;
    int dir = (int)(dt % 2);
    long long b = m->seg_off[tr], e = m->seg_off[tr + 1];
    for (long long kk = 0; kk < e - b; ++kk) {
        long long k = dir ? (e - 1 - kk) : (b + kk);
        long long j = m->seg_fsr[k];
        double l = m->seg_len[k];
        int mm = mat[j];
        for (int g = 0; g < G; ++g) {
            double st = m->sigt[mm * G + g];
            /* Eq. 3: psi_out = psi_in e^{-st l} + qhat (1 - e^{-st l}) */
            double dpsi = (psi[g] - qhat[j * G + g]) * orc_atten(st * l);
            acc[j * G + g] += w * dpsi;
            psi[g] -= dpsi;
        }
    }
}

/* Chains of directed 3D tracks (the successor map followed from a track that
 * no track continues into): the number of such heads, and the longest chain
 * in tracks.  Returns 0, or -3 when some track lies on no chain (a closed
 * loop: every face it meets is reflective) or on more than one. */
static int chain_walk(const struct orc_model *m, long long *heads, long long *n_heads,
                      long long *max_len) {
    const long long ND = 2 * m->n3d;
    char *has_pred = calloc(ND, 1), *seen = calloc(ND, 1);
    long long nh = 0, longest = 0, visited = 0;
    int rc = 0;
    for (long long dt = 0; dt < ND; ++dt)
        if (m->succ[dt] >= 0) has_pred[m->succ[dt]] = 1;
    for (long long dt = 0; dt < ND && rc == 0; ++dt) {
        if (has_pred[dt]) continue;
        if (heads) heads[nh] = dt;
        ++nh;
        long long len = 0;
        for (long long x = dt; x >= 0; x = m->succ[x]) {
            if (seen[x]) { rc = -3; break; }
            seen[x] = 1;
            ++len;
        }
        visited += len;
        if (len > longest) longest = len;
    }
    if (rc == 0 && visited != ND) rc = -3;
    free(has_pred);
    free(seen);
    if (n_heads) *n_heads = nh;
    if (max_len) *max_len = longest;
    return rc;
}

int orc_chain_info(const orc_model *m, long long *n_heads, long long *max_len) {
    if (!m->traced) return -2;
    return chain_walk(m, NULL, n_heads, max_len);
}

int orc_solve(const orc_model *m, const double *q, double tol, int max_iters,
              double *phi_out, double *res_hist, orc_result *res) {
    return orc_solve_ex(m, q, tol, max_iters, 0, 1, phi_out, res_hist, res);
}

int orc_solve_ex(const orc_model *m, const double *q, double tol, int max_iters, int chain,
                 int inner, double *phi_out, double *res_hist, orc_result *res) {
    if (!m->traced) return -2;
    if (inner < 1 || (chain && inner != 1)) return -1;
    long long *heads = NULL, n_heads = 0;
    if (chain) {
        heads = malloc(sizeof(long long) * 2 * (size_t)m->n3d + 8);
        if (chain_walk(m, heads, &n_heads, NULL) != 0) {
            free(heads);
            return -3;
        }
    }
    const int G = m->G;
    const long long NF = m->n_fsr, N3 = m->n3d, ND = 2 * N3;
    const double FOURPI = 4.0 * ORC_PI;
    double *phi = calloc(NF * G, sizeof(double));
    double *qhat = calloc(NF * G, sizeof(double));
    double *psi_a = calloc(ND * G, sizeof(double)), *psi_b = calloc(ND * G, sizeof(double));
    int nth = m->nthreads;
    double *acc_t = calloc((size_t)nth * NF * G, sizeof(double));
    double *tl_leak = calloc(nth, sizeof(double)), *tl_in = calloc(nth, sizeof(double)),
           *tl_out = calloc(nth, sizeof(double));
    int *mat = malloc(sizeof(int) * NF);
    for (long long j = 0; j < NF; ++j) mat[j] = fsr_material(m, j);
    double residual = 1.0;
    int it;
    long long n_sweeps = 0;
    orc_result r;
    memset(&r, 0, sizeof(r));
    for (it = 1; it <= max_iters; ++it) {
        /* reduced source: (scatter + fixed source) / (4 pi Sigma_t), isotropic */
        for (long long j = 0; j < NF; ++j) {
            int mm = mat[j];
            for (int g = 0; g < G; ++g) {
                double s = q[j * G + g];
#if ORC_MUTATION == 2
                for (int gp = 0; gp < G; ++gp) s += m->sigs[(mm * G + g) * G + gp] * phi[j * G + gp];
#else
                for (int gp = 0; gp < G; ++gp) s += m->sigs[(mm * G + gp) * G + g] * phi[j * G + gp];
#endif
                qhat[j * G + g] = s / ((ORC_MUTATION == 1 ? 1.0 : FOURPI) * m->sigt[mm * G + g]);
            }
        }
        /* Lagged mode: each sweep reads the boundary flux the previous
         * sweep left (inner > 1 repeats the sweep with this source, keeping
         * the last sweep's tallies).  Chain mode: every chain is swept from
         * its head (a vacuum face, zero incoming flux) to its end, the
         * outgoing flux of a track entering its successor at once, so no
         * boundary flux is carried between iterations. */
        for (int sw = 0; sw < inner; ++sw) {
        memset(acc_t, 0, sizeof(double) * (size_t)nth * NF * G);
        memset(tl_leak, 0, sizeof(double) * nth);
        memset(tl_in, 0, sizeof(double) * nth);
        memset(tl_out, 0, sizeof(double) * nth);
        ++n_sweeps;
        double *psi_in = (n_sweeps % 2) ? psi_a : psi_b;
        double *psi_out = (n_sweeps % 2) ? psi_b : psi_a;
#pragma omp parallel num_threads(nth)
        {
            int tid = omp_get_thread_num();
            double *acc = acc_t + (size_t)tid * NF * G;
            double psi[64];
            double my_in = 0.0, my_out = 0.0, my_leak = 0.0;
            if (chain) {
#pragma omp for schedule(dynamic, 16)
                for (long long hh = 0; hh < n_heads; ++hh) {
                    for (int g = 0; g < G; ++g) psi[g] = 0.0;
                    for (long long dt = heads[hh]; dt >= 0; dt = m->succ[dt]) {
                        double w = orc_track_weight(m, dt / 2);
                        for (int g = 0; g < G; ++g) my_in += w * psi[g];
                        track_sweep(m, dt, qhat, mat, w, psi, acc);
                        for (int g = 0; g < G; ++g) my_out += w * psi[g];
                        if (m->succ[dt] < 0)
                            for (int g = 0; g < G; ++g) my_leak += w * psi[g];
#if ORC_MUTATION == 9
                        for (int g = 0; g < G; ++g) psi[g] = 0.0;
#endif
                    }
                }
            } else {
#pragma omp for schedule(dynamic, 64)
                for (long long dt = 0; dt < ND; ++dt) {
                    double w = orc_track_weight(m, dt / 2);
                    for (int g = 0; g < G; ++g) { psi[g] = psi_in[dt * G + g]; my_in += w * psi[g]; }
                    track_sweep(m, dt, qhat, mat, w, psi, acc);
                    long long nx = m->succ[dt];
                    for (int g = 0; g < G; ++g) my_out += w * psi[g];
                    if (nx >= 0) {
                        for (int g = 0; g < G; ++g) psi_out[nx * G + g] = psi[g];
                    } else {
                        for (int g = 0; g < G; ++g) my_leak += w * psi[g];
                    }
                }
            }
            tl_in[tid] = my_in; tl_out[tid] = my_out; tl_leak[tid] = my_leak;
        }
        }
        /* Eq. 4 estimator: phi = 4 pi qhat + sum W dpsi / (Sigma_t V) */
        double maxres = 0.0, bal_lhs = 0.0, absorb = 0.0, src = 0.0;
        for (long long j = 0; j < NF; ++j) {
            int mm = mat[j];
            for (int g = 0; g < G; ++g) {
                double a = 0.0;
                for (int t = 0; t < nth; ++t) a += acc_t[(size_t)t * NF * G + j * G + g];
                bal_lhs += a;
                double st = m->sigt[mm * G + g];
                double v = m->vol[j];
                double ph = (ORC_MUTATION == 5 ? 0.0 : FOURPI) * qhat[j * G + g] + (v > 0 ? a / (st * v) : 0.0);
                double old = phi[j * G + g];
                double d = fabs(ph - old);
                double rr = (ph != 0.0) ? d / fabs(ph) : (d == 0.0 ? 0.0 : 1.0);
                if (rr > maxres) maxres = rr;
                phi[j * G + g] = ph;
            }
        }
        for (long long j = 0; j < NF; ++j) {
            int mm = mat[j];
            for (int g = 0; g < G; ++g) {
                double out_scatter = 0.0;
                for (int gp = 0; gp < G; ++gp) out_scatter += m->sigs[(mm * G + g) * G + gp];
                absorb += m->vol[j] * (m->sigt[mm * G + g] - out_scatter) * phi[j * G + g];
                src += m->vol[j] * q[j * G + g];
            }
        }
        double leak = 0, sin_ = 0, sout = 0;
        for (int t = 0; t < nth; ++t) { leak += tl_leak[t]; sin_ += tl_in[t]; sout += tl_out[t]; }
        residual = (it == 1) ? 1.0 : maxres;
        if (res_hist) res_hist[it - 1] = residual;
        r.iters = it; r.residual = residual; r.leakage = leak;
        r.balance_lhs = bal_lhs; r.balance_rhs = sin_ - sout;
        r.absorption = absorb; r.source = src;
        if (residual < tol) break;
    }
    memcpy(phi_out, phi, sizeof(double) * NF * G);
    if (res) *res = r;
    free(phi); free(qhat); free(psi_a); free(psi_b); free(acc_t); free(tl_leak); free(tl_in);
    free(tl_out); free(mat); free(heads);
    return 0;
}

/* ------------------------------------------------------------------ */
/* eigenvalue mode: power iteration on k-eff                           */
/* ------------------------------------------------------------------ */

/* The multiplication factor of the fission-source problem that the paper
 * validates (Table 2 reports k-eff): the isotropic source of group g in FSR j
 * is the scattering term plus chi_g F_j / k, with F_j = sum_g' nuSigma_f,g'
 * phi_j,g' the fission neutron production.  Power iteration, Jacobi in energy
 * like the fixed-source iteration, boundary flux lagged one iteration:
 *   phi = 1, psi = 0, k = 1;
 *   each iteration: qhat from phi and k; one sweep (Eq. 3); phi' by Eq. 4;
 *   P = sum_j V_j F_j(phi), P' = sum_j V_j F_j(phi'); k' = k P' / P;
 *   residual = the larger of |k' - k| / k' and the largest change of the
 *   normalised fission source over FSRs with F_j(phi') > 0,
 *   |F_j(phi') P/P' - F_j(phi)| / (F_j(phi') P/P') (1 at the first
 *   iteration); stop when it falls below tol (after the first iteration) or
 *   at max_iters.
 * The flux is not renormalised between iterations (the 1/k in the source
 * keeps its amplitude bounded), so the boundary flux stays consistent with
 * it.  nu_sigma_f and chi are [M][G]. */
int orc_solve_eigen(const orc_model *m, const double *nu_sigma_f, const double *chi, double tol,
                    int max_iters, double *phi_out, double *k_out, double *res_hist,
                    orc_result *res) {
    if (!m->traced) return -2;
    const int G = m->G;
    const long long NF = m->n_fsr, N3 = m->n3d, ND = 2 * N3;
    const double FOURPI = 4.0 * ORC_PI;
    double *phi = malloc(sizeof(double) * NF * G);
    double *phin = calloc(NF * G, sizeof(double));
    double *qhat = calloc(NF * G, sizeof(double));
    double *fis = calloc(NF, sizeof(double));
    double *psi_a = calloc(ND * G, sizeof(double)), *psi_b = calloc(ND * G, sizeof(double));
    int nth = m->nthreads;
    double *acc_t = calloc((size_t)nth * NF * G, sizeof(double));
    double *tl_leak = calloc(nth, sizeof(double));
    int *mat = malloc(sizeof(int) * NF);
    for (long long j = 0; j < NF; ++j) mat[j] = fsr_material(m, j);
    for (long long i = 0; i < NF * G; ++i) phi[i] = 1.0;
    double k = 1.0, residual = 1.0;
    int it;
    orc_result r;
    memset(&r, 0, sizeof(r));
    for (it = 1; it <= max_iters; ++it) {
        /* fission production of the current flux, and the reduced source */
        double P = 0.0;
        for (long long j = 0; j < NF; ++j) {
            int mm = mat[j];
            double F = 0.0;
            for (int gp = 0; gp < G; ++gp) F += nu_sigma_f[mm * G + gp] * phi[j * G + gp];
            fis[j] = F;
            P += m->vol[j] * F;
            for (int g = 0; g < G; ++g) {
#if ORC_MUTATION == 7
                double s = chi[mm * G + g] * F;
#else
                double s = chi[mm * G + g] * F / k;
#endif
                for (int gp = 0; gp < G; ++gp) s += m->sigs[(mm * G + gp) * G + g] * phi[j * G + gp];
                qhat[j * G + g] = s / (FOURPI * m->sigt[mm * G + g]);
            }
        }
        memset(acc_t, 0, sizeof(double) * (size_t)nth * NF * G);
        memset(tl_leak, 0, sizeof(double) * nth);
        double *psi_in = (it % 2) ? psi_a : psi_b;
        double *psi_out = (it % 2) ? psi_b : psi_a;
#pragma omp parallel num_threads(nth)
        {
            int tid = omp_get_thread_num();
            double *acc = acc_t + (size_t)tid * NF * G;
            double psi[64];
            double my_leak = 0.0;
#pragma omp for schedule(dynamic, 64)
            for (long long dt = 0; dt < ND; ++dt) {
                long long tr = dt / 2;
                int dir = (int)(dt % 2);
                double w = orc_track_weight(m, tr);
                for (int g = 0; g < G; ++g) psi[g] = psi_in[dt * G + g];
                long long b = m->seg_off[tr], e = m->seg_off[tr + 1];
                for (long long kk = 0; kk < e - b; ++kk) {
                    long long kq = dir ? (e - 1 - kk) : (b + kk);
                    long long j = m->seg_fsr[kq];
                    double l = m->seg_len[kq];
                    int mm = mat[j];
                    for (int g = 0; g < G; ++g) {
                        double dpsi = (psi[g] - qhat[j * G + g]) * orc_atten(m->sigt[mm * G + g] * l);
                        acc[j * G + g] += w * dpsi;
                        psi[g] -= dpsi;
                    }
                }
                long long nx = m->succ[dt];
                if (nx >= 0) {
                    for (int g = 0; g < G; ++g) psi_out[nx * G + g] = psi[g];
                } else {
                    for (int g = 0; g < G; ++g) my_leak += w * psi[g];
                }
            }
            tl_leak[tid] = my_leak;
        }
        /* Eq. 4 estimator, the new production and k */
        double Pn = 0.0;
        for (long long j = 0; j < NF; ++j) {
            int mm = mat[j];
            double Fn = 0.0;
            for (int g = 0; g < G; ++g) {
                double a = 0.0;
                for (int t = 0; t < nth; ++t) a += acc_t[(size_t)t * NF * G + j * G + g];
                double v = m->vol[j];
                phin[j * G + g] = FOURPI * qhat[j * G + g] + (v > 0 ? a / (m->sigt[mm * G + g] * v) : 0.0);
                Fn += nu_sigma_f[mm * G + g] * phin[j * G + g];
            }
            Pn += m->vol[j] * Fn;
        }
        double kn = k * Pn / P;
        double maxres = 0.0;
        for (long long j = 0; j < NF; ++j) {
            int mm = mat[j];
            double Fn = 0.0;
            for (int g = 0; g < G; ++g) Fn += nu_sigma_f[mm * G + g] * phin[j * G + g];
            if (Fn > 0.0) {
                double rr = fabs(Fn * (P / Pn) - fis[j]) / (Fn * (P / Pn));
                if (rr > maxres) maxres = rr;
            }
        }
        /* k converges through the boundary flux even where the shape is flat */
        double dk = fabs(kn - k) / fabs(kn);
        if (dk > maxres) maxres = dk;
        memcpy(phi, phin, sizeof(double) * NF * G);
        k = kn;
        double leak = 0.0;
        for (int t = 0; t < nth; ++t) leak += tl_leak[t];
        residual = (it == 1) ? 1.0 : maxres;
        if (res_hist) res_hist[it - 1] = residual;
        r.iters = it; r.residual = residual; r.leakage = leak;
        if (it > 1 && residual < tol) break;
    }
    memcpy(phi_out, phi, sizeof(double) * NF * G);
    if (k_out) *k_out = k;
    if (res) *res = r;
    free(phi); free(phin); free(qhat); free(fis); free(psi_a); free(psi_b); free(acc_t);
    free(tl_leak); free(mat);
    return 0;
}

int orc_sweep_sample(const orc_model *m, long long n_items, const long long *track,
                     const int *dir, const double *qhat, const double *psi_in,
                     double *acc, double *psi_out, long long *n_seg_out) {
    const int G = m->G;
    long long total = 0;
    int bad = 0;
    long long cap = 1 << 16;
    int *f = malloc(sizeof(int) * cap);
    double *l = malloc(sizeof(double) * cap);
    for (long long it = 0; it < n_items; ++it) {
        long long tr = track[it];
        if (tr < 0 || tr >= m->n3d) { bad = 1; break; }
        double p0[3], p1[3], d[3];
        track_endpoints(m, tr, p0, p1, d, NULL, NULL);
        long long ns = trace3d(m, p0, p1, f, l, cap);
        if (ns > cap) { bad = 1; break; }
        total += ns;
        double w = orc_track_weight(m, tr);
        double psi[64];
        for (int g = 0; g < G; ++g) psi[g] = psi_in[it * G + g];
        for (long long kk = 0; kk < ns; ++kk) {
            long long k = dir[it] ? (ns - 1 - kk) : kk;
            long long j = f[k];
            int mm = fsr_material(m, j);
            for (int g = 0; g < G; ++g) {
                double dpsi = (psi[g] - qhat[j * G + g]) * orc_atten(m->sigt[mm * G + g] * l[k]);
                acc[j * G + g] += w * dpsi;
                psi[g] -= dpsi;
            }
        }
        for (int g = 0; g < G; ++g) psi_out[it * G + g] = psi[g];
    }
    free(f); free(l);
    if (n_seg_out) *n_seg_out = total;
    return bad ? -1 : 0;
}
