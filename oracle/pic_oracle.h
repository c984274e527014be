/*
 * pic_oracle.h -- TEST INFRASTRUCTURE, not product code.
 *
 * A plain, slow, single-threaded FP64 CPU implementation of one explicit
 * electromagnetic particle-in-cell step, written from the method description
 * of arXiv:1608.01009 (Section 2: the four stages of the PIC loop -- Maxwell
 * integration, field interpolation, relativistic equations of motion, current
 * deposition; Section 3: double precision, cloud-in-cell form factor,
 * Villasenor-Buneman charge-conserving deposition; Section 4.3: supercells).
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code, header or table with the GPU
 * library; the two meet only through arrays of numbers.
 *
 * Units: c = eps0 = mu0 = 1.  Positions are in cell units, x in [0, n_d).
 * Momenta u = gamma v / c.  Fields are stored on the Yee lattice, x-fastest:
 *   lin(i,j,k) = i + nx*(j + ny*k),
 *   Ex (i+1/2,j,k)  Ey (i,j+1/2,k)  Ez (i,j,k+1/2)
 *   Bx (i,j+1/2,k+1/2)  By (i+1/2,j,k+1/2)  Bz (i+1/2,j+1/2,k)
 *   J_d at the position of E_d; charge density at nodes (i,j,k).
 * All grid indices are periodic.
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int64_t n[3];    /* cells per dimension */
    double dx[3];    /* cell size per dimension (physical units) */
    double dt;       /* time step */
    int64_t S;       /* supercell edge in cells (sort key only) */
    int64_t absorb_x; /* 0: periodic in x; 1: absorbing x boundaries (see below) */
} orc_grid;

/* Absorbing x boundaries (absorb_x = 1; y and z stay periodic).
 *   Lattice: the nodes i = 0 .. n0-1 are inside; the half points i + 1/2 are
 *   inside for i = 0 .. n0-2, and the array slot i = n0-1 of Ex, By, Bz (x =
 *   n0 - 1/2) lies outside and is held at zero.  Lattice points with x index
 *   outside [0, n0) read as zero in the interpolation and receive no current.
 *   Fields: the Yee update of Ey, Ez on the planes i = 0 and i = n0-1 is
 *   replaced by the first-order Mur condition for waves leaving through x,
 *     E^{n+1}[0]    = E^n[1]    + k (E^{n+1}[1]    - E^n[0]),
 *     E^{n+1}[n0-1] = E^n[n0-2] + k (E^{n+1}[n0-2] - E^n[n0-1]),
 *   k = (dt - dx) / (dt + dx) (c = 1); Ex, By, Bz at slot n0-1 stay zero.
 *   Particles live in 0 <= x < n0 - 1.  A move that ends outside deposits
 *   as any move (its current on outside points is dropped; what falls on the
 *   boundary planes x = 0 and x = n0 - 1 meets the Mur-updated Ey, Ez, which
 *   ignore J, and the held-zero slot of Ex), so only its path inside acts;
 *   the particle is removed: marked with x = -1 (its other state as if it
 *   had stayed) and skipped by every later step; the next re-sort drops it.
 *   Sort key of a removed particle: n0 n1 n2 (after every cell). */

/* CIC interpolation of the six field components at one position. */
void orc_gather(const orc_grid* g, const double* const EB[6],
                const double xp[3], double out[6]);

/* Relativistic Boris rotation: u^{n-1/2} -> u^{n+1/2} in place. */
void orc_boris(double q, double m, double dt, const double EB[6], double u[3]);

/* Straight-line position advance x* = x + (dt/dx_d) u_d / gamma (unwrapped). */
void orc_advance(const orc_grid* g, const double u[3], const double x[3],
                 double xs[3]);

/* Villasenor-Buneman deposition of the straight move x0 -> x1 of a particle
 * of charge qw (charge times weight) into J (three Yee arrays). */
void orc_deposit_vb(const orc_grid* g, double* const J[3], const double x0[3],
                    const double x1[3], double qw);

/* Periodic wrap of an advanced position into [0, n_d). */
void orc_wrap(const orc_grid* g, double x[3]);

/* One Yee update: B -= dt/2 curl E; E += dt (curl B - J); B -= dt/2 curl E. */
void orc_fdtd(const orc_grid* g, double* const E[3], double* const B[3],
              const double* const J[3]);

/* Laser source (extension: the injected wave of the laser-plasma benchmark).
 * Adds the soft current sheet Jy += -2 E_L(t) / dx on the node plane x =
 * plane, E_L(t) = E0 sin^2(pi t / T) sin(omega t) for 0 <= t <= T, else 0:
 * in vacuum it radiates Ey = E_L travelling away from the plane on both
 * sides (half the surface current, with c = 1). */
double orc_laser_field(double E0, double omega, double T, double t);
void orc_add_laser(const orc_grid* g, double* Jy, int64_t plane, double E0, double omega,
                   double T, double t);

/* Sort key (supercell-major, then local cell) of one in-domain position. */
int64_t orc_sort_key(const orc_grid* g, const double x[3]);

/* Re-sort of n particles: stable sort by orc_sort_key (every cell's
 * particles together in their previous order, cells grouped by supercell).
 * Permutes the six state arrays and id in place; removed particles
 * (absorbing x) go to the end in their previous order.  Returns the number of
 * particles kept. */
int64_t orc_rebin(const orc_grid* g, int64_t n, double* x, double* y, double* z,
               double* ux, double* uy, double* uz, int64_t* id);

/* Particle loop of one species for one step: gather, Boris, advance,
 * deposit into J (accumulating; J is not cleared here), wrap. */
void orc_push_deposit(const orc_grid* g, double q, double m, double w,
                      int64_t n, double* x, double* y, double* z,
                      double* ux, double* uy, double* uz,
                      const double* const EB[6], double* const J[3]);

/* Mixed-precision variant (integer cell + FP32 offset and FP32 momentum;
 * fields and J FP64).  orc_mixed_round_pos: the position x in [0, n) as
 * stored by the variant (cell + offset rounded to FP32, exactly
 * representable in FP64).  orc_push_deposit_mixed: the particle loop of one
 * species in that arithmetic; positions and momenta are passed as FP64
 * arrays holding values of the variant (as orc_mixed_round_pos and FP32
 * momenta give).  Jabs / Jcnt, when not NULL, accumulate the absolute value
 * and the number of contributions per J node. */
double orc_mixed_round_pos(double x, int64_t n);
void orc_push_deposit_mixed(const orc_grid* g, double q, double m, double w, int64_t n,
                            double* x, double* y, double* z, double* ux, double* uy,
                            double* uz, const double* const EB[6], double* const J[3],
                            double* const* Jabs, int64_t* const* Jcnt);

/* Adjoint of one step (pic_oracle_adjoint.c).  orc_fdtd_adjoint: given the
 * adjoint (lE, lB) of the fields after orc_fdtd, overwrite it with the adjoint
 * of the fields before and write lJ, the adjoint of the current.
 * orc_adjoint_particles: one species' particle loop reversed, from its state
 * (x, u) and the fields at the start of the step; lx..luz hold the adjoint of
 * the state after the step on entry and before it on return; lEB accumulates
 * the adjoint of the interpolated fields. */
void orc_fdtd_adjoint(const orc_grid* g, double* const lE[3], double* const lB[3],
                      double* const lJ[3]);
void orc_adjoint_particles(const orc_grid* g, double q, double m, double w, int64_t n,
                           const double* x, const double* y, const double* z,
                           const double* ux, const double* uy, const double* uz,
                           const double* const EB[6], const double* const lJ[3],
                           double* lx, double* ly, double* lz, double* lux, double* luy,
                           double* luz, double* const lEB[6]);

/* CIC charge density at the nodes: rho += q w W(x-i)W(y-j)W(z-k) / dV. */
void orc_rho(const orc_grid* g, double q, double w, int64_t n,
             const double* x, const double* y, const double* z, double* rho);

/* Gauss residual at the nodes: sum_d (E_d[i] - E_d[i-e_d]) / dx_d - rho. */
void orc_gauss(const orc_grid* g, const double* const E[3], const double* rho,
               double* out);

/* Divergence of B at the cell centres. */
void orc_divb(const orc_grid* g, const double* const B[3], double* out);

/* Kinetic energy sum w m (gamma - 1) of one species. */
double orc_kinetic(double m, double w, int64_t n, const double* ux,
                   const double* uy, const double* uz);

/* Field energy 1/2 sum F^2 dV over ncomp arrays. */
double orc_field_energy(const orc_grid* g, const double* const F[], int ncomp);

#ifdef __cplusplus
}
#endif

#endif
