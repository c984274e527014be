/*
 * pic.h -- C ABI of libpic_hip.so, an MI355X (gfx950) implementation of the
 * explicit electromagnetic particle-in-cell step of arXiv:1608.01009.
 *
 * The step (Section 2 of the paper) has four stages, executed in this order
 * for every step:
 *   1. field interpolation: cloud-in-cell (Section 3) gather of E and B from
 *      the staggered Yee lattice to every particle;
 *   2. relativistic equations of motion: Boris rotation of u = gamma v / c,
 *      then the straight-line position advance x* = x + (dt/dx_d) u_d / gamma;
 *   3. current deposition: Villasenor-Buneman charge-conserving deposition of
 *      the move x -> x* (Section 3), then periodic wrap of x*;
 *   4. Maxwell integration: Yee update B -= dt/2 curl E; E += dt (curl B - J);
 *      B -= dt/2 curl E (B kept at integer time levels).
 * Particles are kept grouped by supercells of S^3 cells (Section 4.3) and are
 * re-sorted every `rebin_every` steps: stably by supercell and cell, then inside
 * each supercell the cells' lists are interleaved in rounds (round r holds the
 * r-th particle of every cell with more than r, cells in x-fastest order).
 *
 * Units: c = eps0 = mu0 = 1.  Positions are in cell units, x_d in [0, n_d).
 * Momenta are u = gamma v / c.  charge q in elementary charges (electron
 * -1), mass m in electron masses, weight w = number of physical particles
 * per macro-particle.  Field arrays are n[0]*n[1]*n[2] doubles, x fastest:
 * lin(i,j,k) = i + n0*(j + n1*k), with the Yee positions
 *   Ex (i+1/2,j,k)  Ey (i,j+1/2,k)  Ez (i,j,k+1/2)
 *   Bx (i,j+1/2,k+1/2)  By (i+1/2,j,k+1/2)  Bz (i+1/2,j+1/2,k)
 *   Jx, Jy, Jz at the positions of Ex, Ey, Ez.
 * y and z are periodic; x is periodic or absorbing (bc_x below).
 *
 * Conventions for every entry point:
 *   - returns a pic_status; nothing throws across the ABI;
 *   - the caller owns every array it passes; the library copies inputs and
 *     writes outputs into caller buffers before returning;
 *   - array pointers may be host memory or device memory of the context's
 *     GPU (the library copies with hipMemcpyDefault);
 *   - a context is used from one thread at a time; all device work goes on
 *     the context's stream;
 *   - on failure, pic_last_error(ctx) describes the cause (pic_last_error
 *     (NULL) after a failed pic_create).
 */
#ifndef PIC_H
#define PIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pic_ctx pic_ctx;

typedef enum {
    PIC_OK = 0,
    PIC_EINVAL = -1,      /* invalid argument or input values */
    PIC_ENOMEM = -2,      /* device or host allocation failed */
    PIC_EDEVICE = -3,     /* a HIP call failed */
    PIC_ECAPACITY = -4,   /* more particles than the species capacity / caller buffer */
    PIC_ENONFINITE = -5,  /* a particle state became NaN or infinite during a step */
    PIC_ESTATE = -6       /* call order violated (e.g. step before any load) */
} pic_status;

/* Arithmetic of the particle loop (gather, push, deposit). */
enum {
    PIC_FP64 = 0,        /* double precision throughout (Section 3 of the paper) */
    PIC_FP32_MIXED = 1   /* positions as integer cell + FP32 offset in [0, 1), FP32 momenta,
                            FP32 gather / Boris / VB split and weights in cell-local
                            coordinates, FP32 J contributions summed in FP64; fields,
                            Yee update and J stay FP64.  Loaded positions are rounded to
                            that form, loaded momenta to FP32; pic_get_particles returns
                            cell + offset exactly.  At most 1024 cells per dimension. */
};

/* Current accumulation.  With deterministic_j = 0 every J contribution is
 * added with FP64 atomics (LDS tile, then global), so J (and through it E, B
 * and the particles) can differ in the last bits from run to run.  With
 * deterministic_j = 1 each FP64 contribution v is split exactly into two
 * integers, hi = rint(v 2^k) and lo = rint((v 2^k - hi) 2^16), summed with
 * integer atomics, and J = hi 2^-k + lo 2^-(k+16): the sums do not depend on
 * the order, so the whole run is bit-reproducible (the scale 2^k is chosen at
 * creation from the capacities and charges so that no sum overflows; each J
 * value carries an error below 2^-(k+17) per contribution, i.e. about 2^-17
 * of the FP64 rounding of the largest possible contribution).  Limit: at most
 * 16383 particles of a species per supercell (PIC_ECAPACITY from pic_step). */

/* Boundaries along x (y and z are always periodic).  The paper's benchmark
 * is periodic; PIC_BC_ABSORBING serves the laser-plasma slab (an extension):
 *   fields: the lattice nodes i = 0 .. n0-1 are inside, the half points
 *     i + 1/2 for i = 0 .. n0-2; the slot i = n0-1 of Ex, By, Bz lies outside
 *     and is held at zero; lattice points outside the box read as zero in the
 *     gather and receive no current; Ey and Ez on the planes i = 0 and
 *     i = n0-1 follow the first-order Mur condition for waves leaving the box,
 *       E^{n+1}[0] = E^n[1] + k (E^{n+1}[1] - E^n[0]),  k = (dt - dx) / (dt + dx),
 *     and the mirror at i = n0-1 (their current is ignored);
 *   particles: live in 0 <= x < n0 - 1; a particle whose move ends outside
 *     deposits that move (only its path inside acts) and is removed: it keeps
 *     its slot with x = -1 until the next re-sort drops it, and the particle
 *     count of the species shrinks then.
 * Requires PIC_FP64 without deterministic_j and supercell 2 or 4 with halo 1
 * or 2, and n0 >= 3; the adjoint does not support it. */
enum {
    PIC_BC_PERIODIC = 0,
    PIC_BC_ABSORBING = 1
};

typedef struct {
    int32_t n[3];           /* cells per dimension; each a multiple of `supercell` */
    int32_t supercell;      /* S: supercell edge in cells (Section 4.3); 1..6 with halo 1,
                               1, 2 or 4 with halo 2 */
    int32_t rebin_every;    /* R >= 1: stable re-sort after every R-th step since the last sort */
    int32_t halo;           /* h: drift margin in cells of the per-supercell LDS tiles; 0 -> 1 */
    int32_t precision;      /* PIC_FP64 or PIC_FP32_MIXED */
    int32_t deterministic_j;  /* 1: bit-reproducible current accumulation (below); 0: FP64
                                 atomics (sums in arbitrary order) */
    int32_t bc_x;           /* PIC_BC_PERIODIC or PIC_BC_ABSORBING */
    int32_t reserved;       /* must be zero */
    void* stream;           /* hipStream_t to run on, or NULL for a library-owned stream */
} pic_grid_t;

typedef struct {
    double charge;          /* q in elementary charges */
    double mass;            /* m in electron masses, > 0 */
    double weight;          /* w > 0: physical particles per macro-particle */
    int64_t capacity;       /* maximum number of particles of this species, < 2^29
                               (each SoA array stays below 4 GiB) */
} pic_species_t;

/* Create a context on the current HIP device.  dx[3] > 0 are the cell sizes,
 * dt > 0 must not exceed the Yee limit 1/sqrt(sum 1/dx_d^2).  Allocates all
 * device memory (particles twice over for the re-sort, E and B twice over for
 * the out-of-place Yee update, currents, sort scratch).  Fields start at
 * zero.  *out receives the context. */
int pic_create(const pic_grid_t* grid, const double dx[3], double dt,
               const pic_species_t* species, int32_t n_species, pic_ctx** out);

/* Replace the particles of one species with n particles (n <= capacity).
 * x, y, z in [0, n_d) (x in [0, n_0 - 1) with PIC_BC_ABSORBING) and finite u
 * are required (PIC_EINVAL otherwise; with PIC_FP32_MIXED also |u| within the
 * FP32 range).
 * id may be NULL (ids 0..n-1).  The particles are re-sorted as described
 * above (their input order breaks ties) and the re-sort counter restarts. */
int pic_load_particles(pic_ctx* ctx, int32_t species, int64_t n,
                       const double* x, const double* y, const double* z,
                       const double* ux, const double* uy, const double* uz,
                       const int64_t* id);

/* Replace E and B (EB[0..5] = Ex, Ey, Ez, Bx, By, Bz); J is cleared. */
int pic_set_fields(pic_ctx* ctx, const double* const EB[6]);

/* Laser source (PIC_BC_ABSORBING contexts; an extension for the laser-plasma
 * slab): every step adds the soft current sheet Jy += -2 E_L(t) / dx_0 on the
 * node plane x = plane (1 <= plane <= n0-2), t = (step + 1/2) dt with `step`
 * the number of steps taken since pic_create, and
 *   E_L(t) = amplitude sin^2(pi t / duration) sin(omega t)  for 0 <= t <= duration,
 * zero otherwise.  In vacuum the sheet radiates a linearly polarised plane
 * wave Ey = E_L travelling away from it on both sides (c = 1); the part
 * towards x = 0 leaves through the absorbing boundary.  In the units here
 * the normalised amplitude a0 gives amplitude = a0 omega.  amplitude = 0
 * switches the source off.  PIC_EINVAL for periodic contexts, a plane out of
 * range or non-finite parameters (duration > 0, omega >= 0). */
int pic_set_laser(pic_ctx* ctx, double amplitude, double omega, double duration,
                  int32_t plane);

/* Advance n_steps >= 0 steps.  Asynchronous on the context stream except for
 * one final 4-byte read of the device error word.  PIC_ENONFINITE if a
 * particle state became non-finite (the state is then unspecified). */
int pic_step(pic_ctx* ctx, int32_t n_steps);

/* Copy Ex, Ey, Ez, Bx, By, Bz, Jx, Jy, Jz (J of the last step) into the nine
 * caller arrays; NULL entries are skipped. */
int pic_get_fields(pic_ctx* ctx, double* const EBJ[9]);

/* Copy the particles of one species, in the library's internal (sorted)
 * order, with their ids.  If capacity < n, returns PIC_ECAPACITY with *n_out
 * set to the number needed.  NULL array pointers are skipped. */
int pic_get_particles(pic_ctx* ctx, int32_t species, int64_t capacity, int64_t* n_out,
                      double* x, double* y, double* z,
                      double* ux, double* uy, double* uz, int64_t* id);

/* Diagnostics of the current state (not part of the timed path):
 * out[0] W_E = 1/2 sum E^2 dV, out[1] W_B, out[2] K = sum w m (gamma - 1),
 * out[3] total charge sum q w (of the particles inside), out[4] max |G - G_ref| with G = div E - rho
 * (CIC rho at the nodes), out[5] max |div B - div B_ref|, out[6] time,
 * out[7] step count.  The references are taken at the first step or
 * diagnostics call after the last load or set_fields. */
int pic_diagnostics(pic_ctx* ctx, double out[8]);

/* Stage timers (HIP events on the context stream), off by default.
 * pic_enable_timers(ctx, mode) resets them and sets the mode: 0 off, 1 every
 * stage below, 2 only the push+deposit kernel in stored order (ms[0]; one
 * event pair per step, which keeps the timing overhead out of the other
 * stages), 3 as 2 on the timed steps 0, 7, 14, ... only (ms[1] counts the
 * launches bracketed; an event pair holds the stream for several
 * microseconds, so sampling keeps that cost out of the step time).  Other
 * modes: PIC_EINVAL. */
int pic_enable_timers(pic_ctx* ctx, int32_t mode);

/* Milliseconds summed over the timed steps, and launch counts:
 *   ms[0] push+deposit kernel (gather, Boris, advance, VB deposit into the
 *         LDS tiles and their flush) reading the particles in stored order,
 *   ms[1] number of those launches,
 *   ms[2] the same kernel on the first step after a re-sort, reading each
 *         particle through the re-sort order (it also writes the new order;
 *         used where supercells hold on average fewer than 1024 particles),
 *   ms[3] number of those launches,
 *   ms[4] far-mover kernel (particles beyond their tile's halo),
 *   ms[5] Yee update, ms[6] re-sort (order computation, and the permutation
 *         of the particle data: of the ids where the push reads through the
 *         order, of every array where supercells hold 1024 or more on
 *         average),
 *   ms[7] total of the pic_step calls, ms[8] number of steps, ms[9] zero. */
int pic_get_timers(pic_ctx* ctx, double ms[10]);

/* Counters: out[0] far movers (particles that were outside their supercell's
 * LDS tile and took the global-memory path), out[1] re-sorts, out[2] steps,
 * out[3] LDS bytes per push+deposit workgroup. */
int pic_get_counters(pic_ctx* ctx, int64_t out[4]);

/* ---- Adjoint (reverse-mode gradient through the step), PIC_FP64 only ----
 *
 * The paper defines the forward step (Section 2: Maxwell integration, field
 * interpolation, equations of motion, current deposition; Section 3: CIC form
 * factor, Villasenor-Buneman deposition); these calls differentiate that
 * step.  The gradient of a scalar L of the current state is carried back to
 * the state at the start of a recorded run:
 *   fields: the transposed Yee update (the curls' transposes, J's -dt);
 *   particles: the vector-Jacobian product of gather, Boris push, advance and
 *     VB deposit (one-sided where a CIC weight or a cell crossing has a kink
 *     at a cell plane), with the transposed interpolation summed with FP64
 *     atomics;
 *   re-sort: each particle's adjoint moves back to its slot before the sort.
 * The forward state of every step is recomputed from checkpoints taken every
 * `checkpoint_every` steps during the recorded run, one segment at a time
 * (memory: one checkpoint per segment, each the particles with ids, E, B and
 * J; plus, during pic_backward, the state of every step of one segment).
 * With deterministic_j the recomputed steps equal the recorded ones bit for
 * bit; with atomic J they may differ by rounding, and the gradient is that of
 * the recomputed trajectory.
 *
 * pic_record: start a recorded run at the current state (any earlier
 * recording is dropped).  The stored particle order at this call, as
 * pic_get_particles returns it now, is the order of the gradient arrays of
 * pic_backward.  checkpoint_every >= 1 (PIC_EINVAL otherwise); PIC_EINVAL
 * for PIC_FP32_MIXED contexts; PIC_ESTATE before any load.  Every pic_step
 * that follows is recorded; pic_load_particles and pic_set_fields end the
 * recording.
 *
 * pic_backward: with seeds dL/d(state now), return dL/d(state at
 * pic_record).  seed_fields[6] (Ex, Ey, Ez, Bx, By, Bz, n_cells values each)
 * and grad_fields[6]: host or device arrays; NULL array or NULL entries mean
 * zero seed / not wanted.  seed_particles and grad_particles: NULL or
 * 6 * n_species pointers, entry [6 s + k] for species s and k = x, y, z, ux,
 * uy, uz, each n_s values, in the current stored order (seeds) and in the
 * stored order at pic_record (gradients); NULL entries as above.  Position
 * gradients are per cell unit (positions are in cell units).  Afterwards the
 * context holds the same state as before the call (particles, fields, J of
 * the last step, counters) and the recording has ended.  PIC_ESTATE without
 * a recording. */
int pic_record(pic_ctx* ctx, int32_t checkpoint_every);
int pic_backward(pic_ctx* ctx, const double* const seed_fields[6],
                 const double* const* seed_particles, double* const grad_fields[6],
                 double* const* grad_particles);

/* ---- Self-check of the push's square root and division ----
 *
 * The relativistic Boris push (Section 2: equations of motion) takes the
 * square root of 1 + |u|^2 and divides by it and by 1 + |t|^2; the library
 * evaluates these with correctly rounded FP64 sequences specialised to those
 * operand ranges (so that positions and momenta are reproducible bit for
 * bit).  This call evaluates the same sequences on arrays, for comparison
 * with any correctly rounded reference:
 *   sq[i] = sqrt(x[i])   for finite x[i] >= 1,
 *   dv[i] = a[i] / b[i]  for 1 <= b[i] < 2^1000 and a[i] = 0 or
 *                        2^-900 < |a[i]| < 2^900;
 * other operands give unspecified values.  n doubles per array, host or
 * device memory (copied to and from device buffers the call allocates and
 * frees).  x and sq NULL: no square roots; a, b and dv NULL: no divisions.
 * PIC_EINVAL for n < 0 or a half-given pair; PIC_ENOMEM / PIC_EDEVICE for HIP
 * failures (message: pic_last_error(NULL)).  Synchronous, on the current
 * device; needs no context. */
int pic_eval_sqrt_div(int64_t n, const double* x, const double* a, const double* b, double* sq,
                      double* dv);

/* The FP32 counterparts used by the PIC_FP32_MIXED push, for comparison with
 * any correctly rounded FP32 reference: sq[i] = sqrt(x[i]) for finite
 * x[i] >= 1; dv[i] = a[i] / b[i] for 1 <= b[i] < 2^64 and a[i] = 0 or
 * 2^-60 < |a[i]| < 2^60 (the push divides h, 2 and 1 by values >= 1;
 * pic_create checks |h| for mixed-precision contexts).  Arrays of n floats,
 * otherwise as pic_eval_sqrt_div. */
int pic_eval_sqrt_div_f32(int64_t n, const float* x, const float* a, const float* b, float* sq,
                          float* dv);

/* pic_eval_sqrt_div for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same results, bit for bit, with the arrays staged through a
 * fixed 8 MiB device buffer that the library holds on each device it runs on
 * until the process ends, instead of buffers allocated per call.  The call
 * makes no hipMalloc / hipFree (the buffer's address is looked up once per
 * device, on the first call with that device current).  n is limited to
 * 209,696 (five arrays of n doubles in 8 MiB): larger n gives PIC_EINVAL with
 * a message (pic_last_error(NULL)).  Calls that overlap on one device share
 * the buffer and race; each call overwrites what it reads. */
int pic_eval_sqrt_div_noalloc(int64_t n, const double* x, const double* a, const double* b,
                              double* sq, double* dv);

/* Message of the last failure on ctx (or of the last failed pic_create or
 * context-free call when ctx is NULL).  Owned by the library; valid until the
 * next call. */
const char* pic_last_error(const pic_ctx* ctx);

/* Release the context and all its device memory.  NULL is ignored. */
void pic_destroy(pic_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif
