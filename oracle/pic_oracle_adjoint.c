/*
 * pic_oracle_adjoint.c -- TEST INFRASTRUCTURE, not product code.
 *
 * Reverse-mode derivative (adjoint) of one step of the FP64 oracle
 * (pic_oracle.c): the transposed Yee update, and per particle the
 * vector-Jacobian product of the chain gather -> Boris -> advance ->
 * Villasenor-Buneman deposit -> wrap.  The paper defines the forward step
 * only (Section 2 stage order, Section 3 schemes); every derivative here is
 * the chain rule applied to the forward formulas of pic_oracle.c, one factor
 * at a time, in the reverse of their order.  Where a forward map has a kink
 * (a cloud-in-cell weight or a cell crossing changes at a cell plane) the
 * derivative is the one-sided one of the piece that contains the point.
 *
 * Only the test suite may load this library.  It shares no code with the
 * GPU library.
 */
#include "pic_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static int64_t awrap(int64_t i, int64_t n) {
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

static int64_t alin(const orc_grid* g, int64_t i, int64_t j, int64_t k) {
    return awrap(i, g->n[0]) + g->n[0] * (awrap(j, g->n[1]) + g->n[1] * awrap(k, g->n[2]));
}

/* ---------------------------------------------------------------------------
 * Transposed Yee update.
 *
 * The forward update is linear in (E, B, J):
 *   B1 = B  - (dt/2) C_E E
 *   E' = E  + dt (C_B B1 - J)
 *   B' = B1 - (dt/2) C_E E'
 * with C_E the forward-difference curl (E lattice -> B lattice) and C_B the
 * backward-difference curl (B lattice -> E lattice).  On the periodic lattice
 * C_B^T = C_E (summation by parts), so the transposed steps, in reverse, are
 *   lE -= (dt/2) C_B lB;   lB += dt C_E lE;   lJ = -dt lE;   lE -= (dt/2) C_B lB.
 * ------------------------------------------------------------------------- */
static void adj_e_from_b(const orc_grid* g, double* const lE[3], double* const lB[3], double coef) {
    const double dx = g->dx[0], dy = g->dx[1], dz = g->dx[2];
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                const int64_t c = alin(g, i, j, k);
                const double cx = (lB[2][c] - lB[2][alin(g, i, j - 1, k)]) / dy -
                                  (lB[1][c] - lB[1][alin(g, i, j, k - 1)]) / dz;
                const double cy = (lB[0][c] - lB[0][alin(g, i, j, k - 1)]) / dz -
                                  (lB[2][c] - lB[2][alin(g, i - 1, j, k)]) / dx;
                const double cz = (lB[1][c] - lB[1][alin(g, i - 1, j, k)]) / dx -
                                  (lB[0][c] - lB[0][alin(g, i, j - 1, k)]) / dy;
                lE[0][c] -= coef * cx;
                lE[1][c] -= coef * cy;
                lE[2][c] -= coef * cz;
            }
}

static void adj_b_from_e(const orc_grid* g, double* const lE[3], double* const lB[3], double coef) {
    const double dx = g->dx[0], dy = g->dx[1], dz = g->dx[2];
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                const int64_t c = alin(g, i, j, k);
                const double cx = (lE[2][alin(g, i, j + 1, k)] - lE[2][c]) / dy -
                                  (lE[1][alin(g, i, j, k + 1)] - lE[1][c]) / dz;
                const double cy = (lE[0][alin(g, i, j, k + 1)] - lE[0][c]) / dz -
                                  (lE[2][alin(g, i + 1, j, k)] - lE[2][c]) / dx;
                const double cz = (lE[1][alin(g, i + 1, j, k)] - lE[1][c]) / dx -
                                  (lE[0][alin(g, i, j + 1, k)] - lE[0][c]) / dy;
                lB[0][c] += coef * cx;
                lB[1][c] += coef * cy;
                lB[2][c] += coef * cz;
            }
}

void orc_fdtd_adjoint(const orc_grid* g, double* const lE[3], double* const lB[3],
                      double* const lJ[3]) {
    const int64_t nc = g->n[0] * g->n[1] * g->n[2];
    adj_e_from_b(g, lE, lB, 0.5 * g->dt);
    adj_b_from_e(g, lE, lB, g->dt);
    for (int d = 0; d < 3; ++d)
        for (int64_t c = 0; c < nc; ++c) lJ[d][c] = -g->dt * lE[d][c];
    adj_e_from_b(g, lE, lB, 0.5 * g->dt);
}

/* ---------------------------------------------------------------------------
 * Cloud-in-cell interpolation and its derivatives.  For component c at
 * position x: lower lattice index i_d and fraction f_d of x_d - s_d (s the
 * Yee stagger), values v[a][b][e] = F[i + (a, b, e)], and
 *   F    = sum w_a(f_x) w_b(f_y) w_e(f_z) v[a][b][e],  w_0 = 1 - f, w_1 = f
 *   dF/dx_d: the same sum with w along d replaced by w'_0 = -1, w'_1 = 1.
 * The value is evaluated as the forward oracle does (nested fused lerps);
 * the derivative as the plain sum.
 * ------------------------------------------------------------------------- */
static const double ASTAG[6][3] = {
    {0.5, 0.0, 0.0}, {0.0, 0.5, 0.0}, {0.0, 0.0, 0.5},
    {0.0, 0.5, 0.5}, {0.5, 0.0, 0.5}, {0.5, 0.5, 0.0},
};

typedef struct {
    int64_t i[3];
    double f[3];
    double v[2][2][2];
} cic_pt;

static void cic_load(const orc_grid* g, const double* F, int c, const double xp[3], cic_pt* p) {
    for (int d = 0; d < 3; ++d) {
        const double xi = xp[d] - ASTAG[c][d];
        const double fl = floor(xi);
        p->i[d] = (int64_t)fl;
        p->f[d] = xi - fl;
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int e = 0; e < 2; ++e)
                p->v[a][b][e] = F[alin(g, p->i[0] + a, p->i[1] + b, p->i[2] + e)];
}

static double cic_value(const cic_pt* p) {
    double r[2];
    for (int e = 0; e < 2; ++e) {
        double q[2];
        for (int b = 0; b < 2; ++b)
            q[b] = fma(p->f[0], p->v[1][b][e] - p->v[0][b][e], p->v[0][b][e]);
        r[e] = fma(p->f[1], q[1] - q[0], q[0]);
    }
    return fma(p->f[2], r[1] - r[0], r[0]);
}

static double wgt(int a, double f) { return a ? f : 1.0 - f; }
static double dwgt(int a) { return a ? 1.0 : -1.0; }

static void cic_grad(const cic_pt* p, double gr[3]) {
    for (int d = 0; d < 3; ++d) gr[d] = 0.0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int e = 0; e < 2; ++e) {
                const double v = p->v[a][b][e];
                gr[0] += dwgt(a) * wgt(b, p->f[1]) * wgt(e, p->f[2]) * v;
                gr[1] += wgt(a, p->f[0]) * dwgt(b) * wgt(e, p->f[2]) * v;
                gr[2] += wgt(a, p->f[0]) * wgt(b, p->f[1]) * dwgt(e) * v;
            }
}

/* transposed interpolation: lF spread over the eight lattice points */
static void cic_scatter(const orc_grid* g, double* F, const cic_pt* p, double lF) {
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int e = 0; e < 2; ++e)
                F[alin(g, p->i[0] + a, p->i[1] + b, p->i[2] + e)] +=
                    lF * wgt(a, p->f[0]) * wgt(b, p->f[1]) * wgt(e, p->f[2]);
}

/* ---------------------------------------------------------------------------
 * Villasenor-Buneman deposit, differentiated.  The deposit of the move
 * x0 -> x1 is a sum over straight segments (A_k, B_k) inside cells c_k; the
 * adjoint needs the gradient of Phi = <lJ, J(x0, x1)>.
 *
 * One segment: with a = A - c, b = B - c, dl = b - a, m = (a + b)/2, and for
 * each current direction d with transverse axes p < r,
 *   Phi_d = jc_d dl_d sum_{bp,br} L[bp][br] (w_bp(m_p) w_br(m_r) + s dl_p dl_r / 12)
 * (s = +1 on the diagonal bp == br, -1 off it; L the lJ_d values of the four
 * edges).  Derivatives in (dl, m), then dPhi/da = -dPhi/ddl + dPhi/dm / 2 and
 * dPhi/db = dPhi/ddl + dPhi/dm / 2.
 *
 * Junctions: the k-th crossing (dimension e_k, plane p_k, time t_k) gives the
 * point P = x0 + t_k (x1 - x0) with P[e_k] = p_k, t_k = (p_k - x0[e_k]) /
 * (x1[e_k] - x0[e_k]); its Jacobian with respect to x0 and x1 is taken by
 * hand below.  The crossings and their order are those of the forward deposit.
 * ------------------------------------------------------------------------- */
static void vb_segment_grad(const orc_grid* g, const double* const lJ[3], const int64_t cell[3],
                            const double A[3], const double B[3], const double jc[3],
                            double gA[3], double gB[3]) {
    double a[3], b[3], dl[3], m[3], gdl[3] = {0, 0, 0}, gm[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) {
        a[d] = A[d] - (double)cell[d];
        b[d] = B[d] - (double)cell[d];
        dl[d] = b[d] - a[d];
        m[d] = 0.5 * (a[d] + b[d]);
    }
    for (int d = 0; d < 3; ++d) {
        const int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
        const int p = e1 < e2 ? e1 : e2;
        const int r = e1 < e2 ? e2 : e1;
        double L[2][2];
        for (int bp = 0; bp < 2; ++bp)
            for (int br = 0; br < 2; ++br) {
                int64_t idx[3] = {cell[0], cell[1], cell[2]};
                idx[p] += bp;
                idx[r] += br;
                L[bp][br] = lJ[d][alin(g, idx[0], idx[1], idx[2])];
            }
        double P = 0.0, dmp = 0.0, dmr = 0.0, K = 0.0;
        for (int bp = 0; bp < 2; ++bp)
            for (int br = 0; br < 2; ++br) {
                const double s = (bp == br) ? 1.0 : -1.0;
                P += L[bp][br] * (wgt(bp, m[p]) * wgt(br, m[r]) + s * dl[p] * dl[r] / 12.0);
                dmp += L[bp][br] * dwgt(bp) * wgt(br, m[r]);
                dmr += L[bp][br] * wgt(bp, m[p]) * dwgt(br);
                K += s * L[bp][br];
            }
        const double f = jc[d] * dl[d];
        gdl[d] += jc[d] * P;
        gm[p] += f * dmp;
        gm[r] += f * dmr;
        gdl[p] += f * K * dl[r] / 12.0;
        gdl[r] += f * K * dl[p] / 12.0;
    }
    for (int d = 0; d < 3; ++d) {
        gA[d] = -gdl[d] + 0.5 * gm[d];
        gB[d] = gdl[d] + 0.5 * gm[d];
    }
}

static void vb_grad(const orc_grid* g, const double* const lJ[3], const double x0[3],
                    const double x1[3], double qw, double gx0[3], double gx1[3]) {
    double jc[3];
    for (int d = 0; d < 3; ++d) {
        const double area = g->dx[(d + 1) % 3] * g->dx[(d + 2) % 3];
        jc[d] = qw / (g->dt * area);
    }
    double dv[3];
    int64_t c0[3], c1[3];
    for (int d = 0; d < 3; ++d) {
        dv[d] = x1[d] - x0[d];
        c0[d] = (int64_t)floor(x0[d]);
        c1[d] = (int64_t)floor(x1[d]);
    }
    int nc = 0;
    double tc[3], pc[3];
    int dc[3];
    for (int d = 0; d < 3; ++d)
        if (c1[d] != c0[d]) {
            const double p = (double)(c0[d] > c1[d] ? c0[d] : c1[d]);
            tc[nc] = (p - x0[d]) / dv[d];
            pc[nc] = p;
            dc[nc] = d;
            ++nc;
        }
    for (int i = 1; i < nc; ++i) {
        int j = i;
        while (j > 0 && tc[j - 1] > tc[j]) {
            double tt = tc[j]; tc[j] = tc[j - 1]; tc[j - 1] = tt;
            double pp = pc[j]; pc[j] = pc[j - 1]; pc[j - 1] = pp;
            int dd = dc[j]; dc[j] = dc[j - 1]; dc[j - 1] = dd;
            --j;
        }
    }
    /* points P[0] = x0, P[k+1] = junction k, P[nc+1] = x1; segment k from
     * P[k] to P[k+1] in cell cells[k] */
    double P[5][3], gP[5][3];
    int64_t cells[4][3];
    for (int d = 0; d < 3; ++d) {
        P[0][d] = x0[d];
        P[nc + 1][d] = x1[d];
        cells[0][d] = c0[d];
    }
    for (int k = 0; k < nc; ++k) {
        for (int d = 0; d < 3; ++d) P[k + 1][d] = x0[d] + tc[k] * dv[d];
        P[k + 1][dc[k]] = pc[k];
        for (int d = 0; d < 3; ++d) cells[k + 1][d] = cells[k][d];
        cells[k + 1][dc[k]] = c1[dc[k]];
    }
    memset(gP, 0, sizeof(gP));
    for (int k = 0; k <= nc; ++k) {
        double gA[3], gB[3];
        vb_segment_grad(g, lJ, cells[k], P[k], P[k + 1], jc, gA, gB);
        for (int d = 0; d < 3; ++d) {
            gP[k][d] += gA[d];
            gP[k + 1][d] += gB[d];
        }
    }
    for (int d = 0; d < 3; ++d) {
        gx0[d] += gP[0][d];
        gx1[d] += gP[nc + 1][d];
    }
    for (int k = 0; k < nc; ++k) {
        const int e = dc[k];
        const double t = tc[k];
        /* Jacobian rows of the junction point: dP[f]/dx0, dP[f]/dx1 */
        for (int f = 0; f < 3; ++f) {
            if (f == e) continue;                 /* P[e] = plane: constant */
            const double G = gP[k + 1][f];
            gx0[f] += G * (1.0 - t);
            gx1[f] += G * t;
            gx0[e] += G * dv[f] * (t - 1.0) / dv[e];
            gx1[e] += G * dv[f] * (-t) / dv[e];
        }
    }
}

/* ---------------------------------------------------------------------------
 * One species, one step, reversed.  Inputs: the state (x, u) at the start of
 * the step, the fields E/B at the start of the step, lJ = dPhi/dJ of the
 * step's current; lx, lu hold the adjoint of the particle state at the end of
 * the step and are overwritten with the adjoint at the start; lEB accumulates
 * the transposed interpolation.  Boris (forward, pic_oracle.c):
 *   um = u + h E; gm = sqrt(1 + |um|^2); hg = h / gm; t = hg B;
 *   sf = 2 / (1 + |t|^2); s = sf t; up = um + um x t; upl = um + up x s;
 *   u1 = upl + h E;  x* = x + (dt/dx) u1 / gamma(u1);  J += VB(x, x*);
 *   x' = wrap(x*) (derivative 1).
 * ------------------------------------------------------------------------- */
static double dot3(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static void cross3(const double a[3], const double b[3], double out[3]) {
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

void orc_adjoint_particles(const orc_grid* g, double q, double m, double w, int64_t n,
                           const double* x, const double* y, const double* z,
                           const double* ux, const double* uy, const double* uz,
                           const double* const EB[6], const double* const lJ[3],
                           double* lx, double* ly, double* lz, double* lux, double* luy,
                           double* luz, double* const lEB[6]) {
    const double h = (q * g->dt) / (2.0 * m);
    const double qw = q * w;
    for (int64_t p = 0; p < n; ++p) {
        const double x0[3] = {x[p], y[p], z[p]};
        const double u0[3] = {ux[p], uy[p], uz[p]};
        /* forward values */
        cic_pt cp[6];
        double F[6], dF[6][3];
        for (int c = 0; c < 6; ++c) {
            cic_load(g, EB[c], c, x0, &cp[c]);
            F[c] = cic_value(&cp[c]);
            cic_grad(&cp[c], dF[c]);
        }
        const double* E = F;
        const double* B = F + 3;
        double um[3], t[3], s[3], up[3], upl[3], u1[3];
        for (int d = 0; d < 3; ++d) um[d] = fma(h, E[d], u0[d]);
        const double gm = sqrt(fma(um[2], um[2], fma(um[1], um[1], fma(um[0], um[0], 1.0))));
        const double hg = h / gm;
        for (int d = 0; d < 3; ++d) t[d] = hg * B[d];
        const double sf = 2.0 / fma(t[2], t[2], fma(t[1], t[1], fma(t[0], t[0], 1.0)));
        for (int d = 0; d < 3; ++d) s[d] = sf * t[d];
        for (int d = 0; d < 3; ++d) {
            const int e = (d + 1) % 3, f = (d + 2) % 3;
            up[d] = fma(um[e], t[f], fma(-um[f], t[e], um[d]));
        }
        for (int d = 0; d < 3; ++d) {
            const int e = (d + 1) % 3, f = (d + 2) % 3;
            upl[d] = fma(up[e], s[f], fma(-up[f], s[e], um[d]));
        }
        for (int d = 0; d < 3; ++d) u1[d] = fma(h, E[d], upl[d]);
        double x1[3];
        orc_advance(g, u1, x0, x1);
        const double gi = 1.0 / sqrt(fma(u1[2], u1[2], fma(u1[1], u1[1], fma(u1[0], u1[0], 1.0))));

        /* reverse */
        double lxs[3] = {lx[p], ly[p], lz[p]};          /* wrap: derivative 1 */
        double lu1[3] = {lux[p], luy[p], luz[p]};
        double gx0[3] = {0, 0, 0}, gx1[3] = {0, 0, 0};
        vb_grad(g, lJ, x0, x1, qw, gx0, gx1);
        for (int d = 0; d < 3; ++d) lxs[d] += gx1[d];
        double lx0[3];
        for (int d = 0; d < 3; ++d) lx0[d] = lxs[d] + gx0[d];
        /* x* = x0 + (dt/dx) u1 gi:  d(u_d gi)/du_e = gi delta_de - u_d u_e gi^3 */
        double v[3];
        for (int d = 0; d < 3; ++d) v[d] = (g->dt / g->dx[d]) * lxs[d];
        const double uv = dot3(u1, v);
        for (int d = 0; d < 3; ++d) lu1[d] += gi * v[d] - u1[d] * uv * gi * gi * gi;
        /* Boris, reversed */
        double lE[3], lB[3], lupl[3], lum[3], lup[3], ls[3], lt[3], tmp[3];
        for (int d = 0; d < 3; ++d) {
            lE[d] = h * lu1[d];                           /* u1 = upl + h E */
            lupl[d] = lu1[d];
        }
        for (int d = 0; d < 3; ++d) lum[d] = lupl[d];     /* upl = um + up x s */
        cross3(s, lupl, lup);
        cross3(lupl, up, ls);
        for (int d = 0; d < 3; ++d) lum[d] += lup[d];     /* up = um + um x t */
        cross3(t, lup, tmp);
        for (int d = 0; d < 3; ++d) lum[d] += tmp[d];
        cross3(lup, um, lt);
        const double lst = dot3(ls, t);                   /* s = sf t */
        for (int d = 0; d < 3; ++d) lt[d] += sf * ls[d] - sf * sf * lst * t[d];
        for (int d = 0; d < 3; ++d) lB[d] = hg * lt[d];   /* t = hg B */
        const double lhg = dot3(lt, B);
        const double lgm = -(hg / gm) * lhg;              /* hg = h / gm */
        for (int d = 0; d < 3; ++d) lum[d] += (lgm / gm) * um[d];   /* gm = sqrt(1+|um|^2) */
        double lu0[3];
        for (int d = 0; d < 3; ++d) {
            lu0[d] = lum[d];                              /* um = u0 + h E */
            lE[d] += h * lum[d];
        }
        /* interpolation, reversed */
        const double lF[6] = {lE[0], lE[1], lE[2], lB[0], lB[1], lB[2]};
        for (int c = 0; c < 6; ++c) {
            for (int d = 0; d < 3; ++d) lx0[d] += lF[c] * dF[c][d];
            cic_scatter(g, lEB[c], &cp[c], lF[c]);
        }
        lx[p] = lx0[0];
        ly[p] = lx0[1];
        lz[p] = lx0[2];
        lux[p] = lu0[0];
        luy[p] = lu0[1];
        luz[p] = lu0[2];
    }
}
