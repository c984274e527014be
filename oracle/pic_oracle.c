/*
 * pic_oracle.c -- TEST INFRASTRUCTURE, not product code.
 *
 * Plain single-threaded FP64 reference of the explicit electromagnetic PIC
 * step of arXiv:1608.01009.  The paper names the stages (Section 2) and the
 * schemes (Section 3: double precision, cloud-in-cell form factor,
 * Villasenor-Buneman charge-conserving deposition) but prints no formula;
 * every formula below is the textbook definition of the named scheme, coded
 * directly, with no blocking, fusion or reordering.  Build with
 * -ffp-contract=off so that every expression rounds as written.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code with the GPU library.
 */
#include "pic_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Yee stagger of the six field components, in cell units (Section 2 names
 * the field solver only; the Yee lattice is the standard staggered grid). */
static const double STAG[6][3] = {
    {0.5, 0.0, 0.0}, /* Ex */
    {0.0, 0.5, 0.0}, /* Ey */
    {0.0, 0.0, 0.5}, /* Ez */
    {0.0, 0.5, 0.5}, /* Bx */
    {0.5, 0.0, 0.5}, /* By */
    {0.5, 0.5, 0.0}, /* Bz */
};

static int64_t wrapi(int64_t i, int64_t n) {
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

static int64_t lin(const orc_grid* g, int64_t i, int64_t j, int64_t k) {
    return wrapi(i, g->n[0]) + g->n[0] * (wrapi(j, g->n[1]) + g->n[1] * wrapi(k, g->n[2]));
}

/* ---------------------------------------------------------------------------
 * Field interpolation with the cloud-in-cell form factor (Section 2 stage 2,
 * Section 3 form factor).  Each component is interpolated trilinearly from the
 * eight nearest points of its own staggered lattice:
 *   xi_d = x_d - s_d, i_d = floor(xi_d), f_d = xi_d - i_d,
 * as nested linear interpolation, first along x, then y, then z:
 *   lerp(a, b, f) = a + f (b - a), evaluated as fma(f, b - a, a),
 * which equals sum_{a,b,c} w_a(f_x) w_b(f_y) w_c(f_z) F[i+a, j+b, k+c] with
 * w_0(f) = 1 - f, w_1(f) = f.
 * ------------------------------------------------------------------------- */
static double lerp(double a, double b, double f) { return fma(f, b - a, a); }

/* lattice value; with absorbing x boundaries points outside 0 <= i < n0 are 0 */
static double fetch(const orc_grid* g, const double* F, int64_t i, int64_t j, int64_t k) {
    if (g->absorb_x && (i < 0 || i >= g->n[0])) return 0.0;
    return F[lin(g, i, j, k)];
}

void orc_gather(const orc_grid* g, const double* const EB[6], const double xp[3],
                double out[6]) {
    for (int c = 0; c < 6; ++c) {
        int64_t i[3];
        double f[3];
        for (int d = 0; d < 3; ++d) {
            double xi = xp[d] - STAG[c][d];
            double fl = floor(xi);
            i[d] = (int64_t)fl;
            f[d] = xi - fl;
        }
        double fz[2];
        for (int cc = 0; cc < 2; ++cc) {
            double fy[2];
            for (int b = 0; b < 2; ++b) {
                double f0 = fetch(g, EB[c], i[0], i[1] + b, i[2] + cc);
                double f1 = fetch(g, EB[c], i[0] + 1, i[1] + b, i[2] + cc);
                fy[b] = lerp(f0, f1, f[0]);
            }
            fz[cc] = lerp(fy[0], fy[1], f[1]);
        }
        out[c] = lerp(fz[0], fz[1], f[2]);
    }
}

/* ---------------------------------------------------------------------------
 * Relativistic equations of motion (Section 2), advanced with the Boris
 * scheme: half electric kick, magnetic rotation, half electric kick.
 *   h = q dt / (2 m)
 *   u- = u + h E;  gamma- = sqrt(1 + |u-|^2)
 *   t = (h / gamma-) B;  s = 2 t / (1 + |t|^2)
 *   u' = u- + u- x t;  u+ = u- + u' x s;  u_new = u+ + h E
 * The paper fixes no evaluation order.  Each sum of products is evaluated
 * as a chain of fused multiply-adds (one rounding per product-add):
 *   1 + |v|^2          = fma(v2, v2, fma(v1, v1, fma(v0, v0, 1)))
 *   a0 + (b1 c2 - b2 c1) = fma(b1, c2, fma(-b2, c1, a0))   (cross products)
 *   u + h E            = fma(h, E, u)
 * ------------------------------------------------------------------------- */
static double one_plus_sq(const double v[3]) {
    return fma(v[2], v[2], fma(v[1], v[1], fma(v[0], v[0], 1.0)));
}

/* a + b x c, component d, as two fused multiply-adds */
static double add_cross(const double a[3], const double b[3], const double c[3], int d) {
    const int e = (d + 1) % 3, f = (d + 2) % 3;
    return fma(b[e], c[f], fma(-b[f], c[e], a[d]));
}

void orc_boris(double q, double m, double dt, const double EB[6], double u[3]) {
    const double h = (q * dt) / (2.0 * m);
    const double* E = EB;
    const double* B = EB + 3;
    double um[3], t[3], s[3], up[3], upl[3];
    for (int d = 0; d < 3; ++d) um[d] = fma(h, E[d], u[d]);
    double gm = sqrt(one_plus_sq(um));
    double hg = h / gm;
    for (int d = 0; d < 3; ++d) t[d] = hg * B[d];
    double sf = 2.0 / one_plus_sq(t);
    for (int d = 0; d < 3; ++d) s[d] = sf * t[d];
    for (int d = 0; d < 3; ++d) up[d] = add_cross(um, um, t, d);   /* u' = u- + u- x t */
    for (int d = 0; d < 3; ++d) upl[d] = add_cross(um, up, s, d);  /* u+ = u- + u' x s */
    for (int d = 0; d < 3; ++d) u[d] = fma(h, E[d], upl[d]);
}

/* x*_d = x_d + ((dt/dx_d) u_d) g,  g = 1 / sqrt(1 + |u|^2); unwrapped; the
 * final product-add is fused. */
void orc_advance(const orc_grid* g, const double u[3], const double x[3], double xs[3]) {
    double gi = 1.0 / sqrt(one_plus_sq(u));
    for (int d = 0; d < 3; ++d) {
        double cdt = g->dt / g->dx[d];
        xs[d] = fma(cdt * u[d], gi, x[d]);
    }
}

/* If x >= L subtract L, else if x < 0 add L; a result equal to L becomes 0
 * (L and 0 are the same point of the periodic lattice). */
void orc_wrap(const orc_grid* g, double x[3]) {
    for (int d = 0; d < 3; ++d) {
        double L = (double)g->n[d];
        double v = x[d];
        if (v >= L)
            v = v - L;
        else if (v < 0.0)
            v = v + L;
        if (v == L) v = 0.0;
        x[d] = v;
    }
}

/* ---------------------------------------------------------------------------
 * Villasenor-Buneman charge-conserving current deposition (Section 3).
 *
 * The straight move x0 -> x1 is cut at every cell plane it crosses.  Inside a
 * cell with integer corner c, a segment from A to B (local a = A - c,
 * b = B - c, delta = b - a, mid m = (a + b)/2) carries the charge flux
 *   Jx[c_x, c_y+beta, c_z+gam] += jc_x * delta_x * W_{beta,gam}(y, z)
 *   W_00 = (1-m_y)(1-m_z) + dy dz/12    W_10 = m_y (1-m_z) - dy dz/12
 *   W_01 = (1-m_y) m_z   - dy dz/12     W_11 = m_y m_z     + dy dz/12
 * (dy, dz here the local displacements), i.e. the time integral of the
 * velocity times the CIC transverse weights along the segment;
 * jc_x = qw / (dt * area of the x face).  Jy and Jz follow by permuting axes.
 *
 * Crossing order: dimension d crosses plane p_d = max(floor x0_d, floor x1_d)
 * at t_d = (p_d - x0_d) / (x1_d - x0_d); crossings are taken in increasing
 * t, ties in dimension order x, y, z.  Each junction point is computed once
 * as x0 + t_k (x1 - x0) with its crossing coordinate set to p_d exactly, and
 * serves as the end of one segment and the start of the next.
 * ------------------------------------------------------------------------- */
static void vb_segment(const orc_grid* g, double* const J[3], const int64_t cell[3],
                       const double A[3], const double B[3], const double jc[3]) {
    double a[3], b[3], dl[3], m[3];
    for (int d = 0; d < 3; ++d) {
        a[d] = A[d] - (double)cell[d];
        b[d] = B[d] - (double)cell[d];
        dl[d] = b[d] - a[d];
        m[d] = 0.5 * (a[d] + b[d]);
    }
    for (int d = 0; d < 3; ++d) {
        int e1 = (d + 1) % 3; /* first transverse axis */
        int e2 = (d + 2) % 3; /* second transverse axis */
        /* the two transverse axes in increasing dimension order */
        int p = e1 < e2 ? e1 : e2;
        int r = e1 < e2 ? e2 : e1;
        double cross = (dl[p] * dl[r]) / 12.0;
        double flux = jc[d] * dl[d];
        for (int bp = 0; bp < 2; ++bp) {
            double wp = bp ? m[p] : 1.0 - m[p];
            for (int br = 0; br < 2; ++br) {
                double wr = br ? m[r] : 1.0 - m[r];
                double W = wp * wr + ((bp == br) ? cross : -cross);
                int64_t idx[3] = {cell[0], cell[1], cell[2]};
                idx[p] += bp;
                idx[r] += br;
                if (g->absorb_x && (idx[0] < 0 || idx[0] >= g->n[0])) continue;
                J[d][lin(g, idx[0], idx[1], idx[2])] += flux * W;
            }
        }
    }
}

void orc_deposit_vb(const orc_grid* g, double* const J[3], const double x0[3],
                    const double x1[3], double qw) {
    double jc[3];
    for (int d = 0; d < 3; ++d) {
        double area = g->dx[(d + 1) % 3] * g->dx[(d + 2) % 3];
        jc[d] = qw / (g->dt * area);
    }
    double dv[3];
    int64_t c0[3], c1[3];
    for (int d = 0; d < 3; ++d) {
        dv[d] = x1[d] - x0[d];
        c0[d] = (int64_t)floor(x0[d]);
        c1[d] = (int64_t)floor(x1[d]);
    }
    /* crossings, collected in dimension order, then stably sorted by time */
    int nc = 0;
    double tc[3], pc[3];
    int dc[3];
    for (int d = 0; d < 3; ++d) {
        if (c1[d] != c0[d]) {
            double p = (double)(c0[d] > c1[d] ? c0[d] : c1[d]);
            tc[nc] = (p - x0[d]) / dv[d];
            pc[nc] = p;
            dc[nc] = d;
            ++nc;
        }
    }
    for (int i = 1; i < nc; ++i) { /* stable insertion sort on tc */
        int j = i;
        while (j > 0 && tc[j - 1] > tc[j]) {
            double tt = tc[j]; tc[j] = tc[j - 1]; tc[j - 1] = tt;
            double pp = pc[j]; pc[j] = pc[j - 1]; pc[j - 1] = pp;
            int dd = dc[j]; dc[j] = dc[j - 1]; dc[j - 1] = dd;
            --j;
        }
    }
    double A[3] = {x0[0], x0[1], x0[2]};
    int64_t cell[3] = {c0[0], c0[1], c0[2]};
    for (int k = 0; k <= nc; ++k) {
        double B[3];
        if (k < nc) {
            for (int d = 0; d < 3; ++d) B[d] = x0[d] + tc[k] * dv[d];
            B[dc[k]] = pc[k];
        } else {
            for (int d = 0; d < 3; ++d) B[d] = x1[d];
        }
        vb_segment(g, J, cell, A, B, jc);
        if (k < nc) {
            for (int d = 0; d < 3; ++d) A[d] = B[d];
            cell[dc[k]] = c1[dc[k]];
        }
    }
}

/* ---------------------------------------------------------------------------
 * Maxwell integration (Section 2 stage 1) with the Yee scheme, B kept at
 * integer time levels by splitting its leapfrog update into two halves.
 *   (curl E)_x[i,j,k] = (Ez[i,j+1,k]-Ez[i,j,k])/dy - (Ey[i,j,k+1]-Ey[i,j,k])/dz
 *   (curl B)_x[i,j,k] = (Bz[i,j,k]-Bz[i,j-1,k])/dy - (By[i,j,k]-By[i,j,k-1])/dz
 * and cyclic permutations.
 * ------------------------------------------------------------------------- */
static void half_b(const orc_grid* g, double* const E[3], double* const B[3]) {
    const int64_t nx = g->n[0], ny = g->n[1], nz = g->n[2];
    const double dx = g->dx[0], dy = g->dx[1], dz = g->dx[2];
    const double hdt = 0.5 * g->dt;
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t c = lin(g, i, j, k);
                double cx = (E[2][lin(g, i, j + 1, k)] - E[2][c]) / dy -
                            (E[1][lin(g, i, j, k + 1)] - E[1][c]) / dz;
                double cy = (E[0][lin(g, i, j, k + 1)] - E[0][c]) / dz -
                            (E[2][lin(g, i + 1, j, k)] - E[2][c]) / dx;
                double cz = (E[1][lin(g, i + 1, j, k)] - E[1][c]) / dx -
                            (E[0][lin(g, i, j + 1, k)] - E[0][c]) / dy;
                B[0][c] = B[0][c] - hdt * cx;
                B[1][c] = B[1][c] - hdt * cy;
                B[2][c] = B[2][c] - hdt * cz;
            }
}

static void full_e(const orc_grid* g, double* const E[3], double* const B[3],
                   const double* const J[3]) {
    const int64_t nx = g->n[0], ny = g->n[1], nz = g->n[2];
    const double dx = g->dx[0], dy = g->dx[1], dz = g->dx[2];
    const double dt = g->dt;
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t c = lin(g, i, j, k);
                double cx = (B[2][c] - B[2][lin(g, i, j - 1, k)]) / dy -
                            (B[1][c] - B[1][lin(g, i, j, k - 1)]) / dz;
                double cy = (B[0][c] - B[0][lin(g, i, j, k - 1)]) / dz -
                            (B[2][c] - B[2][lin(g, i - 1, j, k)]) / dx;
                double cz = (B[1][c] - B[1][lin(g, i - 1, j, k)]) / dx -
                            (B[0][c] - B[0][lin(g, i, j - 1, k)]) / dy;
                E[0][c] = E[0][c] + dt * (cx - J[0][c]);
                E[1][c] = E[1][c] + dt * (cy - J[1][c]);
                E[2][c] = E[2][c] + dt * (cz - J[2][c]);
            }
}

/* Absorbing x boundaries: the same updates on the inside points, the slot
 * n0-1 of Ex, By, Bz held at zero, Mur on Ey, Ez at i = 0 and i = n0-1. */
static void half_b_abs(const orc_grid* g, double* const E[3], double* const B[3]) {
    const int64_t nx = g->n[0], ny = g->n[1], nz = g->n[2];
    const double dx = g->dx[0], dy = g->dx[1], dz = g->dx[2];
    const double hdt = 0.5 * g->dt;
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t c = lin(g, i, j, k);
                double cx = (E[2][lin(g, i, j + 1, k)] - E[2][c]) / dy -
                            (E[1][lin(g, i, j, k + 1)] - E[1][c]) / dz;
                B[0][c] = B[0][c] - hdt * cx;
                if (i == nx - 1) {
                    B[1][c] = 0.0;
                    B[2][c] = 0.0;
                    continue;
                }
                double cy = (E[0][lin(g, i, j, k + 1)] - E[0][c]) / dz -
                            (E[2][lin(g, i + 1, j, k)] - E[2][c]) / dx;
                double cz = (E[1][lin(g, i + 1, j, k)] - E[1][c]) / dx -
                            (E[0][lin(g, i, j + 1, k)] - E[0][c]) / dy;
                B[1][c] = B[1][c] - hdt * cy;
                B[2][c] = B[2][c] - hdt * cz;
            }
}

static void full_e_abs(const orc_grid* g, double* const E[3], double* const B[3],
                       const double* const J[3]) {
    const int64_t nx = g->n[0], ny = g->n[1], nz = g->n[2];
    const double dx = g->dx[0], dy = g->dx[1], dz = g->dx[2];
    const double dt = g->dt;
    const double kmur = (dt - dx) / (dt + dx);
    /* old values that the Mur condition needs */
    const size_t plane = (size_t)(ny * nz);
    double* old = (double*)malloc(8 * plane * sizeof(double));
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j) {
            const size_t q = (size_t)(j + ny * k);
            for (int d = 1; d < 3; ++d) {
                old[(4 * (d - 1) + 0) * plane + q] = E[d][lin(g, 0, j, k)];
                old[(4 * (d - 1) + 1) * plane + q] = E[d][lin(g, 1, j, k)];
                old[(4 * (d - 1) + 2) * plane + q] = E[d][lin(g, nx - 1, j, k)];
                old[(4 * (d - 1) + 3) * plane + q] = E[d][lin(g, nx - 2, j, k)];
            }
        }
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t c = lin(g, i, j, k);
                if (i < nx - 1) {
                    double cx = (B[2][c] - B[2][lin(g, i, j - 1, k)]) / dy -
                                (B[1][c] - B[1][lin(g, i, j, k - 1)]) / dz;
                    E[0][c] = E[0][c] + dt * (cx - J[0][c]);
                } else {
                    E[0][c] = 0.0;
                }
                if (i == 0 || i == nx - 1) continue;       /* Mur below */
                double cy = (B[0][c] - B[0][lin(g, i, j, k - 1)]) / dz -
                            (B[2][c] - B[2][lin(g, i - 1, j, k)]) / dx;
                double cz = (B[1][c] - B[1][lin(g, i - 1, j, k)]) / dx -
                            (B[0][c] - B[0][lin(g, i, j - 1, k)]) / dy;
                E[1][c] = E[1][c] + dt * (cy - J[1][c]);
                E[2][c] = E[2][c] + dt * (cz - J[2][c]);
            }
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j) {
            const size_t q = (size_t)(j + ny * k);
            for (int d = 1; d < 3; ++d) {
                const double e0 = old[(4 * (d - 1) + 0) * plane + q];
                const double e1 = old[(4 * (d - 1) + 1) * plane + q];
                const double eN = old[(4 * (d - 1) + 2) * plane + q];
                const double eN1 = old[(4 * (d - 1) + 3) * plane + q];
                E[d][lin(g, 0, j, k)] = e1 + kmur * (E[d][lin(g, 1, j, k)] - e0);
                E[d][lin(g, nx - 1, j, k)] = eN1 + kmur * (E[d][lin(g, nx - 2, j, k)] - eN);
            }
        }
    free(old);
}

void orc_fdtd(const orc_grid* g, double* const E[3], double* const B[3],
              const double* const J[3]) {
    if (g->absorb_x) {
        half_b_abs(g, E, B);
        full_e_abs(g, E, B, J);
        half_b_abs(g, E, B);
        return;
    }
    half_b(g, E, B);
    full_e(g, E, B, J);
    half_b(g, E, B);
}

double orc_laser_field(double E0, double omega, double T, double t) {
    const double pi = 3.14159265358979323846;
    if (!(t >= 0.0 && t <= T)) return 0.0;
    const double env = sin(pi * t / T);
    return E0 * (env * env) * sin(omega * t);
}

void orc_add_laser(const orc_grid* g, double* Jy, int64_t plane, double E0, double omega,
                   double T, double t) {
    const double s = (-2.0 * orc_laser_field(E0, omega, T, t)) / g->dx[0];
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j) {
            const int64_t c = lin(g, plane, j, k);
            Jy[c] = Jy[c] + s;
        }
}

/* ---------------------------------------------------------------------------
 * Per-cell particle storage grouped by supercells (Sections 3 and 4.3).
 *
 * The key orders particles by supercell (x-fastest over supercells), then by
 * cell inside the supercell (x-fastest).  A stable sort on that key stores
 * every cell's particles together, in their previous order, and the cells of
 * a supercell next to each other: the per-cell lists of the paper, laid out
 * supercell by supercell.
 * ------------------------------------------------------------------------- */
int64_t orc_sort_key(const orc_grid* g, const double x[3]) {
    const int64_t S = g->S;
    if (g->absorb_x && x[0] < 0.0) return g->n[0] * g->n[1] * g->n[2];   /* removed */
    int64_t c[3];
    for (int d = 0; d < 3; ++d) c[d] = (int64_t)floor(x[d]);
    int64_t ns0 = g->n[0] / S, ns1 = g->n[1] / S;
    int64_t sc = c[0] / S + ns0 * (c[1] / S + ns1 * (c[2] / S));
    int64_t loc = c[0] % S + S * (c[1] % S + S * (c[2] % S));
    return sc * S * S * S + loc;
}

static void permute_d(double* a, const int64_t* perm, int64_t n, double* tmp) {
    for (int64_t i = 0; i < n; ++i) tmp[i] = a[perm[i]];
    memcpy(a, tmp, (size_t)n * sizeof(double));
}

int64_t orc_rebin(const orc_grid* g, int64_t n, double* x, double* y, double* z,
                  double* ux, double* uy, double* uz, int64_t* id) {
    if (n <= 0) return 0;
    const int64_t ncell = g->n[0] * g->n[1] * g->n[2];
    const int64_t nkeys = ncell + (g->absorb_x ? 1 : 0);   /* key ncell: removed */
    int64_t* key = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    int64_t* start = (int64_t*)calloc((size_t)nkeys + 1, sizeof(int64_t));
    int64_t* perm = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    double* tmp = (double*)malloc((size_t)n * sizeof(double));
    int64_t* itmp = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    /* stable counting sort by key */
    for (int64_t p = 0; p < n; ++p) {
        double xp[3] = {x[p], y[p], z[p]};
        key[p] = orc_sort_key(g, xp);
        start[key[p] + 1] += 1;
    }
    for (int64_t k = 0; k < nkeys; ++k) start[k + 1] += start[k];   /* first slot of each key */
    const int64_t kept = start[ncell];          /* removed particles sort after every cell */
    for (int64_t p = 0; p < n; ++p) perm[start[key[p]]++] = p;     /* previous order kept */
    permute_d(x, perm, n, tmp);
    permute_d(y, perm, n, tmp);
    permute_d(z, perm, n, tmp);
    permute_d(ux, perm, n, tmp);
    permute_d(uy, perm, n, tmp);
    permute_d(uz, perm, n, tmp);
    for (int64_t i = 0; i < n; ++i) itmp[i] = id[perm[i]];
    memcpy(id, itmp, (size_t)n * sizeof(int64_t));
    free(key); free(start); free(perm); free(tmp); free(itmp);
    return kept;
}

/* One species' particle loop for one step, in array order (Section 2: field
 * interpolation and equations of motion form the push; the deposit follows). */
void orc_push_deposit(const orc_grid* g, double q, double m, double w, int64_t n,
                      double* x, double* y, double* z, double* ux, double* uy,
                      double* uz, const double* const EB[6], double* const J[3]) {
    const double qw = q * w;
    for (int64_t p = 0; p < n; ++p) {
        double x0[3] = {x[p], y[p], z[p]};
        double u[3] = {ux[p], uy[p], uz[p]};
        double f[6];
        double x1[3];
        if (g->absorb_x && x0[0] < 0.0) continue;       /* removed earlier */
        orc_gather(g, EB, x0, f);
        orc_boris(q, m, g->dt, f, u);
        orc_advance(g, u, x0, x1);
        orc_deposit_vb(g, J, x0, x1, qw);
        orc_wrap(g, x1);
        /* absorbing x: a particle that ends outside 0 <= x < n0 - 1 is removed
         * (its current on outside points was dropped; the part on the
         * boundary planes meets the Mur-updated Ey, Ez, which ignore J) */
        if (g->absorb_x && !(x1[0] >= 0.0 && x1[0] < (double)(g->n[0] - 1))) x1[0] = -1.0;
        x[p] = x1[0]; y[p] = x1[1]; z[p] = x1[2];
        ux[p] = u[0]; uy[p] = u[1]; uz[p] = u[2];
    }
}

/* ---------------------------------------------------------------------------
 * Diagnostics (not part of the step).
 * ------------------------------------------------------------------------- */
void orc_rho(const orc_grid* g, double q, double w, int64_t n, const double* x,
             const double* y, const double* z, double* rho) {
    const double dv = g->dx[0] * g->dx[1] * g->dx[2];
    const double qv = (q * w) / dv;
    for (int64_t p = 0; p < n; ++p) {
        double xp[3] = {x[p], y[p], z[p]};
        int64_t i[3];
        double f[3];
        if (g->absorb_x && xp[0] < 0.0) continue;        /* removed */
        for (int d = 0; d < 3; ++d) {
            double fl = floor(xp[d]);
            i[d] = (int64_t)fl;
            f[d] = xp[d] - fl;
        }
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int c = 0; c < 2; ++c) {
                    double w3 = (a ? f[0] : 1.0 - f[0]) * (b ? f[1] : 1.0 - f[1]) *
                                (c ? f[2] : 1.0 - f[2]);
                    rho[lin(g, i[0] + a, i[1] + b, i[2] + c)] += qv * w3;
                }
    }
}

void orc_gauss(const orc_grid* g, const double* const E[3], const double* rho, double* out) {
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                int64_t c = lin(g, i, j, k);
                double dive = (E[0][c] - E[0][lin(g, i - 1, j, k)]) / g->dx[0] +
                              (E[1][c] - E[1][lin(g, i, j - 1, k)]) / g->dx[1] +
                              (E[2][c] - E[2][lin(g, i, j, k - 1)]) / g->dx[2];
                out[c] = dive - rho[c];
            }
}

void orc_divb(const orc_grid* g, const double* const B[3], double* out) {
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                int64_t c = lin(g, i, j, k);
                out[c] = (B[0][lin(g, i + 1, j, k)] - B[0][c]) / g->dx[0] +
                         (B[1][lin(g, i, j + 1, k)] - B[1][c]) / g->dx[1] +
                         (B[2][lin(g, i, j, k + 1)] - B[2][c]) / g->dx[2];
            }
}

double orc_kinetic(double m, double w, int64_t n, const double* ux, const double* uy,
                   const double* uz) {
    double s = 0.0;
    /* gamma - 1 = u^2 / (1 + sqrt(1 + u^2)), free of the cancellation of
     * sqrt(1 + u^2) - 1 for slow particles */
    for (int64_t p = 0; p < n; ++p) {
        double u2 = (ux[p] * ux[p] + uy[p] * uy[p]) + uz[p] * uz[p];
        s += u2 / (1.0 + sqrt(1.0 + u2));
    }
    return w * m * s;
}

double orc_field_energy(const orc_grid* g, const double* const F[], int ncomp) {
    const int64_t nc = g->n[0] * g->n[1] * g->n[2];
    const double dv = g->dx[0] * g->dx[1] * g->dx[2];
    double s = 0.0;
    for (int c = 0; c < ncomp; ++c)
        for (int64_t i = 0; i < nc; ++i) s += F[c][i] * F[c][i];
    return 0.5 * s * dv;
}

/* ---------------------------------------------------------------------------
 * Mixed-precision variant of the particle loop (an extension beyond the
 * paper, which computes in double precision throughout, Section 3).
 *
 * A position is stored as an integer cell c_d and an FP32 offset o_d in
 * [0, 1) (x_d = c_d + o_d exactly), the momentum as three FP32 values.  The
 * step performs the FP64 scheme's operations in FP32 arithmetic (every
 * operation rounded to single precision; fused multiply-adds where the FP64
 * scheme has them), with cell-local coordinates:
 *   gather:  per component and axis with stagger 1/2: i = c, f = o - 1/2 if
 *            o >= 1/2, else i = c - 1, f = o + 1/2; stagger 0: i = c, f = o;
 *            field values rounded to FP32, nested lerps x, y, z;
 *   Boris:   as orc_boris with h = (float)(q dt / 2m);
 *   advance: o* = fma((float)(dt/dx_d) u_d, g, o) with g = 1/sqrt(1+|u|^2),
 *            relative to the cell corner (so o* lies in (-1, 2));
 *   deposit: the VB split and segment weights of orc_deposit_vb in FP32 in
 *            cell-local coordinates, jc_d = (float)(q w / (dt area_d)); each
 *            segment contribution is added to the FP64 J;
 *   cell:    s = floor(o*), c = (c + s) mod n, o = o* - s; an offset that
 *            rounds to 1 becomes 0 in the next cell.
 * The fields, the Yee update and J stay FP64.  Jabs and Jcnt (optional)
 * receive the sum of |contribution| and the number of contributions per J
 * node, which bound the effect of summing the FP32 contributions in another
 * order or precision.
 * ------------------------------------------------------------------------- */
static float lerpf_(float a, float b, float f) { return fmaf(f, b - a, a); }

/* cell and FP32 offset of a position x in [0, n): x - c is exact in FP64 */
static void split_pos(double x, int64_t n, int64_t* c, float* o) {
    double fl = floor(x);
    int64_t ci = (int64_t)fl;
    float of = (float)(x - fl);
    if (of >= 1.0f) {
        of = 0.0f;
        ci = ci + 1 == n ? 0 : ci + 1;
    }
    *c = ci;
    *o = of;
}

double orc_mixed_round_pos(double x, int64_t n) {
    int64_t c;
    float o;
    split_pos(x, n, &c, &o);
    return (double)c + (double)o;
}

static void gather_mixed(const orc_grid* g, const double* const EB[6], const int64_t c[3],
                         const float o[3], float out[6]) {
    for (int comp = 0; comp < 6; ++comp) {
        int64_t i[3];
        float f[3];
        for (int d = 0; d < 3; ++d) {
            if (STAG[comp][d] != 0.0) {
                if (o[d] >= 0.5f) {
                    i[d] = c[d];
                    f[d] = o[d] - 0.5f;
                } else {
                    i[d] = c[d] - 1;
                    f[d] = o[d] + 0.5f;
                }
            } else {
                i[d] = c[d];
                f[d] = o[d];
            }
        }
        float fz[2];
        for (int cc = 0; cc < 2; ++cc) {
            float fy[2];
            for (int b = 0; b < 2; ++b) {
                float f0 = (float)EB[comp][lin(g, i[0], i[1] + b, i[2] + cc)];
                float f1 = (float)EB[comp][lin(g, i[0] + 1, i[1] + b, i[2] + cc)];
                fy[b] = lerpf_(f0, f1, f[0]);
            }
            fz[cc] = lerpf_(fy[0], fy[1], f[1]);
        }
        out[comp] = lerpf_(fz[0], fz[1], f[2]);
    }
}

static float one_plus_sqf(const float v[3]) {
    return fmaf(v[2], v[2], fmaf(v[1], v[1], fmaf(v[0], v[0], 1.0f)));
}

static float add_crossf(const float a[3], const float b[3], const float c[3], int d) {
    const int e = (d + 1) % 3, f = (d + 2) % 3;
    return fmaf(b[e], c[f], fmaf(-b[f], c[e], a[d]));
}

static void boris_mixed(float h, const float EB[6], float u[3]) {
    const float* E = EB;
    const float* B = EB + 3;
    float um[3], t[3], s[3], up[3], upl[3];
    for (int d = 0; d < 3; ++d) um[d] = fmaf(h, E[d], u[d]);
    float gm = sqrtf(one_plus_sqf(um));
    float hg = h / gm;
    for (int d = 0; d < 3; ++d) t[d] = hg * B[d];
    float sf = 2.0f / one_plus_sqf(t);
    for (int d = 0; d < 3; ++d) s[d] = sf * t[d];
    for (int d = 0; d < 3; ++d) up[d] = add_crossf(um, um, t, d);
    for (int d = 0; d < 3; ++d) upl[d] = add_crossf(um, up, s, d);
    for (int d = 0; d < 3; ++d) u[d] = fmaf(h, E[d], upl[d]);
}

static void add_j(const orc_grid* g, double* const J[3], double* const* Jabs, int64_t* const* Jcnt,
                  int d, int64_t i, int64_t j, int64_t k, float v) {
    int64_t n = lin(g, i, j, k);
    J[d][n] += (double)v;
    if (Jabs) Jabs[d][n] += fabs((double)v);
    if (Jcnt) Jcnt[d][n] += 1;
}

/* one segment A -> B (cell-local coordinates relative to the start cell's
 * corner) inside the cell with relative corner rc; cell = start cell */
static void vb_segment_mixed(const orc_grid* g, double* const J[3], double* const* Jabs,
                             int64_t* const* Jcnt, const int64_t cell[3], const int rc[3],
                             const float A[3], const float B[3], const float jc[3]) {
    float a[3], b[3], dl[3], m[3];
    for (int d = 0; d < 3; ++d) {
        a[d] = A[d] - (float)rc[d];
        b[d] = B[d] - (float)rc[d];
        dl[d] = b[d] - a[d];
        m[d] = 0.5f * (a[d] + b[d]);
    }
    for (int d = 0; d < 3; ++d) {
        int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
        int p = e1 < e2 ? e1 : e2;
        int r = e1 < e2 ? e2 : e1;
        float cross = (dl[p] * dl[r]) / 12.0f;
        float flux = jc[d] * dl[d];
        for (int bp = 0; bp < 2; ++bp) {
            float wp = bp ? m[p] : 1.0f - m[p];
            for (int br = 0; br < 2; ++br) {
                float wr = br ? m[r] : 1.0f - m[r];
                float W = wp * wr + ((bp == br) ? cross : -cross);
                int64_t idx[3] = {cell[0] + rc[0], cell[1] + rc[1], cell[2] + rc[2]};
                idx[p] += bp;
                idx[r] += br;
                add_j(g, J, Jabs, Jcnt, d, idx[0], idx[1], idx[2], flux * W);
            }
        }
    }
}

static void deposit_mixed(const orc_grid* g, double* const J[3], double* const* Jabs,
                          int64_t* const* Jcnt, const int64_t cell[3], const float o0[3],
                          const float o1[3], const float jc[3]) {
    float dv[3];
    int c1[3];
    for (int d = 0; d < 3; ++d) {
        dv[d] = o1[d] - o0[d];
        c1[d] = (int)floorf(o1[d]);
    }
    int nc = 0;
    float tc[3], pc[3];
    int dc[3];
    for (int d = 0; d < 3; ++d) {
        if (c1[d] != 0) {
            float p = (float)(c1[d] > 0 ? c1[d] : 0);
            tc[nc] = (p - o0[d]) / dv[d];
            pc[nc] = p;
            dc[nc] = d;
            ++nc;
        }
    }
    for (int i = 1; i < nc; ++i) {
        int j = i;
        while (j > 0 && tc[j - 1] > tc[j]) {
            float tt = tc[j]; tc[j] = tc[j - 1]; tc[j - 1] = tt;
            float pp = pc[j]; pc[j] = pc[j - 1]; pc[j - 1] = pp;
            int dd = dc[j]; dc[j] = dc[j - 1]; dc[j - 1] = dd;
            --j;
        }
    }
    float A[3] = {o0[0], o0[1], o0[2]};
    int rc[3] = {0, 0, 0};
    for (int k = 0; k <= nc; ++k) {
        float B[3];
        if (k < nc) {
            for (int d = 0; d < 3; ++d) B[d] = fmaf(tc[k], dv[d], o0[d]);
            B[dc[k]] = pc[k];
        } else {
            for (int d = 0; d < 3; ++d) B[d] = o1[d];
        }
        vb_segment_mixed(g, J, Jabs, Jcnt, cell, rc, A, B, jc);
        if (k < nc) {
            for (int d = 0; d < 3; ++d) A[d] = B[d];
            rc[dc[k]] = c1[dc[k]];
        }
    }
}

void orc_push_deposit_mixed(const orc_grid* g, double q, double m, double w, int64_t n,
                            double* x, double* y, double* z, double* ux, double* uy,
                            double* uz, const double* const EB[6], double* const J[3],
                            double* const* Jabs, int64_t* const* Jcnt) {
    const float h = (float)((q * g->dt) / (2.0 * m));
    float cdt[3], jc[3];
    for (int d = 0; d < 3; ++d) {
        cdt[d] = (float)(g->dt / g->dx[d]);
        double area = g->dx[(d + 1) % 3] * g->dx[(d + 2) % 3];
        jc[d] = (float)((q * w) / (g->dt * area));
    }
    double* X[3] = {x, y, z};
    double* U[3] = {ux, uy, uz};
    for (int64_t p = 0; p < n; ++p) {
        int64_t c[3];
        float o[3], u[3], f[6], o1[3];
        for (int d = 0; d < 3; ++d) {
            split_pos(X[d][p], g->n[d], &c[d], &o[d]);
            u[d] = (float)U[d][p];
        }
        gather_mixed(g, EB, c, o, f);
        boris_mixed(h, f, u);
        float gi = 1.0f / sqrtf(one_plus_sqf(u));
        for (int d = 0; d < 3; ++d) o1[d] = fmaf(cdt[d] * u[d], gi, o[d]);
        deposit_mixed(g, J, Jabs, Jcnt, c, o, o1, jc);
        for (int d = 0; d < 3; ++d) {
            float s = floorf(o1[d]);
            int64_t cn = wrapi(c[d] + (int64_t)s, g->n[d]);
            float on = o1[d] - s;
            if (on >= 1.0f) {
                on = 0.0f;
                cn = cn + 1 == g->n[d] ? 0 : cn + 1;
            }
            X[d][p] = (double)cn + (double)on;
            U[d][p] = (double)u[d];
        }
    }
}
