// Internal declarations shared by the HIP translation units of libpic_hip.so.
// Device code targets gfx950 (CDNA4): wave64, 160 KiB LDS per CU, native
// FP64 atomics in LDS (ds_add_f64) and in global memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

// Device error word bits.
enum : unsigned {
    ERR_NONFINITE = 1u,   // a particle state became NaN / Inf during a step
    ERR_BADPOS = 2u,      // a loaded position is outside [0, n) or not finite
    ERR_DETCAP = 4u,      // deterministic J: a supercell holds more than kDetMaxPerSupercell
    ERR_SORT = 8u,        // internal: the neighbourhood re-sort found inconsistent counts
};

// Deterministic current accumulation.  Every FP64 contribution v is split
// exactly into two integers, hi = rint(v 2^k) and lo = rint((v 2^k - hi)
// 2^kDetLoBits), so that v = hi 2^-k + lo 2^-(k + kDetLoBits) up to
// 2^-(k + kDetLoBits + 1); hi and lo are summed with integer atomics (in the
// LDS tiles: hi in 64 bits, lo in 32 bits; in global memory both in 64
// bits), which gives the same sums in any order.  k is chosen per context
// so that no hi sum can overflow; a supercell may hold at most
// kDetMaxPerSupercell particles so that no LDS lo sum can overflow (a
// particle adds at most four contributions, one per VB segment, to a node).
constexpr int kDetLoBits = 16;
constexpr int kDetMaxPerSupercell = 16383;

struct DetJ {
    unsigned long long* hi[3];  // global accumulators (two's complement sums)
    long long* lo[3];
    double scale;               // 2^k
};

__device__ __forceinline__ void det_split(double v, double scale, unsigned long long& hi, int& lo) {
#pragma clang fp contract(off)
    const double t = v * scale;          // exact: scale is a power of two
    const double h = __builtin_rint(t);
    const double r = t - h;              // exact: |r| <= 1/2 and r is t's fraction
    hi = (unsigned long long)(long long)h;
    lo = (int)__builtin_rint(r * (double)(1 << kDetLoBits));
}

// Geometry and constants of one context, passed by value to kernels.
struct Geom {
    int n[3];          // cells
    int ncell;         // n0*n1*n2
    int S;             // supercell edge
    int ns[3];         // supercells per dimension
    int nsc;           // number of supercells
    int h;             // halo (drift margin) of the LDS tiles, cells
    double dt;
    double cdt[3];     // dt / dx_d
    double dx[3];
    int absorb_x;      // 1: absorbing x boundaries (Mur fields, particle removal)
};

// Per-species constants of the particle push.
struct SpeciesC {
    double q, m, w;
    double hq;         // q dt / (2 m)
    double jc[3];      // q w / (dt * face area of the d face)
};

// SoA particle arrays of one species (one buffer of the double buffer).
struct Parts {
    double* x;
    double* y;
    double* z;
    double* ux;
    double* uy;
    double* uz;
    int64_t* id;
    unsigned spare = 0;   // index of a writable slot past the last particle (x .. uz)
};

struct Fields {
    double* E[3];
    double* B[3];
};

// Mixed-precision variant: per-species FP32 constants and the packed particle
// arrays (cell = i | j << 10 | k << 20, offsets in [0, 1), momenta).
struct SpeciesM {
    float h;           // (float)(q dt / (2 m))
    float jc[3];       // (float)(q w / (dt * face area of the d face))
    float cdt[3];      // (float)(dt / dx_d)
};

struct PartsM {
    unsigned* cell;
    float* ox;
    float* oy;
    float* oz;
    float* ux;
    float* uy;
    float* uz;
    int64_t* id;
    unsigned spare = 0;   // index of a writable slot past the last particle (cell .. uz)
};

// ---- launchers (implemented in the kernel translation units) --------------

// Gather + Boris + advance + VB deposit + wrap for every particle of one
// species; deposits are accumulated into J (which must hold the sum of the
// previous species of this step, or zero).  Particle i of the new order is
// read from src at perm[i] (or at i when perm is NULL) and written to dst at
// i (dst may equal src when perm is NULL).  keys, when not NULL, receives the
// sort key of every particle's new position.  Particles outside their
// supercell's tile are appended to far_q (capacity >= particles; counter
// far_n, zero on entry) and left to launch_far_movers, which must follow
// with the same arguments.
hipError_t launch_push_deposit(const Geom& g, const SpeciesC& sp, const Parts& src,
                               const Parts& dst, const unsigned* perm, unsigned* keys,
                               const int* sc_off, const Fields& f, double* const J[3],
                               unsigned* err, unsigned long long* nfar, int* far_q,
                               unsigned* far_n, unsigned* far_n_next, const DetJ& det,
                               hipStream_t s);
// The particles queued by launch_push_deposit, through global memory; clears
// far_n_next (the counter of the next launch).
hipError_t launch_far_movers(const Geom& g, const SpeciesC& sp, const Parts& src,
                             const Parts& dst, const unsigned* perm, unsigned* keys,
                             const Fields& f, double* const J[3], unsigned* err,
                             unsigned long long* nfar, int* far_q, unsigned* far_n,
                             unsigned* far_n_next, const DetJ& det, hipStream_t s);
// det.hi[0] != NULL selects the deterministic accumulation into det (J is
// then not touched; see launch_j_from_fixed).
// Two species in one launch (arrays of two for every per-species argument):
// one E/B tile load and one J flush per supercell for both, each species with
// its own far-mover queue and counters; both read through a re-sort order or
// neither.  Not with the deterministic J (push_deposit_pair_supported).
bool push_deposit_pair_supported(int S, int h, bool det);
hipError_t launch_push_deposit_pair(const Geom& g, const SpeciesC* sp, const Parts* src,
                                    const Parts* dst, const unsigned* const* perm,
                                    unsigned* const* keys, const int* const* sc_off,
                                    const Fields& f, double* const J[3], unsigned* err,
                                    unsigned long long* nfar, int* const* far_q,
                                    unsigned* const* far_n, unsigned* const* far_n_next,
                                    const DetJ& det, hipStream_t s);
int push_deposit_lds_bytes(const Geom& g, bool det);
bool push_deposit_supported(int S, int h);

// Mixed-precision counterparts of launch_push_deposit / launch_far_movers
// (same contracts, packed particle arrays, FP32 tiles and arithmetic).
hipError_t launch_push_mixed(const Geom& g, const SpeciesM& sp, const PartsM& src,
                             const PartsM& dst, const unsigned* perm, unsigned* keys,
                             const int* sc_off, const Fields& f, double* const J[3],
                             unsigned* err, unsigned long long* nfar, int* far_q,
                             unsigned* far_n, unsigned* far_n_next, const DetJ& det,
                             hipStream_t s);
hipError_t launch_far_mixed(const Geom& g, const SpeciesM& sp, const PartsM& src,
                            const PartsM& dst, const unsigned* perm, unsigned* keys,
                            const Fields& f, double* const J[3], unsigned* err,
                            unsigned long long* nfar, int* far_q, unsigned* far_n,
                            unsigned* far_n_next, const DetJ& det, hipStream_t s);
int push_mixed_lds_bytes(const Geom& g, bool det);
// FP64 positions / momenta (device arrays x, y, z, ux, uy, uz) -> packed
// arrays and sort keys; ERR_BADPOS for positions outside [0, n), non-finite
// values or momenta beyond FP32 range.
hipError_t launch_to_mixed(const Geom& g, int64_t n, const double* const x[6], const PartsM& dst,
                           unsigned* keys, unsigned* err, hipStream_t s);
// packed arrays -> FP64 positions (cell + offset, exact) and momenta
hipError_t launch_to_double(int64_t n, const PartsM& src, double* const x[6], hipStream_t s);
// dst[i] = src[perm[i]] for the packed arrays and the ids
hipError_t launch_permute_mixed(int64_t n, const unsigned* perm, const PartsM& src,
                                const PartsM& dst, hipStream_t s);

// Deterministic mode: J = hi 2^-k + lo 2^-(k + kDetLoBits) for the three
// components, then the accumulators are cleared.
hipError_t launch_j_from_fixed(int64_t n, const DetJ& det, double* const J[3], hipStream_t s);

// Yee update from the fields f into fo (distinct arrays); also clears Jclear
// (the buffer the next step deposits into).
hipError_t launch_fdtd(const Geom& g, const Fields& f, const Fields& fo, double* const J[3],
                       double* const Jclear[3], hipStream_t s);

// The same update with absorbing x boundaries (Mur planes, outside slots
// held at zero) and the laser sheet: laser_j is added to Jy on the node plane
// laser_plane (-1: none) and kept in J.
hipError_t launch_fdtd_absorbing(const Geom& g, const Fields& f, const Fields& fo,
                                 double* const J[3], double* const Jclear[3], int laser_plane,
                                 double laser_j, hipStream_t s);

// Fill n doubles with zero.
hipError_t launch_zero(double* p, int64_t n, hipStream_t s);

// Re-sort order of one species: perm (new index -> current index) and the
// supercell offsets of the new order.  keys == NULL: computed from src's
// positions, with ERR_BADPOS set for positions outside [0, n) or non-finite
// values.  scratch must hold rebin_scratch_bytes(n, g) bytes.
size_t rebin_scratch_bytes(int64_t n, const Geom& g);
hipError_t launch_sort(const Geom& g, int64_t n, const unsigned* keys, const Parts& src,
                       unsigned* perm, int* sc_off, void* scratch, unsigned* err, hipStream_t s);
// Particle arrays that a re-sort moves into the new order: count arrays of
// 4- or 8-byte elements, src in the current order, dst another buffer.
struct MoveArrays {
    const void* src[8];
    void* dst[8];
    int bytes[8];
    int count = 0;
};
// The same order for a re-sort after a push (keys from that push, old_off the
// supercell offsets of the current order), computed per supercell from its
// 27 neighbours' particles when every particle's new supercell is one of the
// 27 around its old one (periodic x, S^3 <= 64), after launch_resort_prep.
// The classification raises *far_host (coherent pinned host memory, cleared
// here; far_dev is its device address) if
// any particle moved farther, and the rest of the re-sort is queued behind it,
// each of its kernels doing nothing in that case; the host then waits for the
// classification (event ev, recorded here).  *done is false (nothing else
// written) when there are any,
// or the grid is not supported, and launch_sort must be used instead.  With
// move (count > 0) the arrays are also written in the new order
// (dst[i] = src[perm[i]]), staged per supercell through LDS.
// Start of every re-sort: sc_prev = sc_off (the supercell offsets of the
// order before it) and the neighbourhood re-sort's counters in scratch
// cleared, in one launch.
hipError_t launch_resort_prep(const Geom& g, int64_t n, const int* sc_off, int* sc_prev,
                              void* scratch, hipStream_t s);
hipError_t launch_sort_local(const Geom& g, int64_t n, const unsigned* keys, const int* old_off,
                             unsigned* perm, int* sc_off, void* scratch, unsigned* err,
                             const MoveArrays* move, unsigned* far_host, unsigned* far_dev,
                             hipEvent_t ev, hipStream_t s, bool* done);
// dst[i] = src[perm[i]] for the six state arrays and the ids.
hipError_t launch_permute(int64_t n, const unsigned* perm, const Parts& src, const Parts& dst,
                          hipStream_t s);
hipError_t launch_permute_ids(int64_t n, const unsigned* perm, const int64_t* src, int64_t* dst,
                              hipStream_t s);
// dst[i] = src[perm[i]] for the arrays of mv, for a re-sort whose old order had
// the supercell offsets old_off (each supercell's particles, mostly in one old
// block, are staged through LDS); new_off: the offsets of the new order.
// skip (device, may be null): nothing is done if *skip != 0 when the launch runs.
hipError_t launch_staged_permute(const Geom& g, int64_t n, const unsigned* perm, const int* old_off,
                                const int* new_off, const MoveArrays& mv, hipStream_t s,
                                const unsigned* skip = nullptr);

// Adjoint of one step (FP64).  launch_fdtd_adjoint: the transposed Yee update
// in place on (lE, lB), writing lJ (the adjoint of the step's current).
// launch_particle_adjoint: one species' particle loop reversed from its state
// at the start of the step (state = x, y, z, ux, uy, uz) and the fields at the
// start of the step; lam (six arrays) holds the adjoint of the state after the
// step on entry and before it on return; lEB accumulates the transposed
// interpolation with atomics.  launch_unpermute: dst[perm[i]] = src[i] for six
// arrays (the adjoint of a re-sort).
hipError_t launch_fdtd_adjoint(const Geom& g, double* const lE[3], double* const lB[3],
                               double* const lJ[3], hipStream_t s);
hipError_t launch_particle_adjoint(const Geom& g, const SpeciesC& sp, int64_t n,
                                   const double* const state[6], const double* const EB[6],
                                   const double* const lJ[3], double* const lam[6],
                                   double* const lEB[6], hipStream_t s);
hipError_t launch_unpermute(int64_t n, const unsigned* perm, double* const src[6],
                            double* const dst[6], hipStream_t s);

// The push's correctly rounded square root (x >= 1) and division (divisor in
// [1, 2^1000)) on device arrays; sq or dv NULL skips that part.
hipError_t launch_sqrt_div(int64_t n, const double* x, const double* a, const double* b,
                           double* sq, double* dv, hipStream_t s);
// The same for the mixed-precision push's FP32 square root (x >= 1) and
// division (divisor in [1, 2^64), numerator 0 or of magnitude in
// (2^-60, 2^60)).
hipError_t launch_sqrt_div_f32(int64_t n, const float* x, const float* a, const float* b,
                               float* sq, float* dv, hipStream_t s);

// Diagnostics.
hipError_t launch_sum_squares(const double* const a[3], int64_t n, double* acc, hipStream_t s);
// kinetic sum of gamma - 1; with x given, particles with x < 0 (removed) are
// skipped and the others counted into cnt
hipError_t launch_kinetic(const double* ux, const double* uy, const double* uz, int64_t n,
                          double* acc, hipStream_t s, const double* x = nullptr,
                          double* cnt = nullptr);
hipError_t launch_rho(const Geom& g, double qv, const double* x, const double* y,
                      const double* z, int64_t n, double* rho, hipStream_t s);
hipError_t launch_gauss(const Geom& g, const Fields& f, const double* rho, double* out,
                        hipStream_t s);
hipError_t launch_divb(const Geom& g, const Fields& f, double* out, hipStream_t s);
hipError_t launch_maxabs_diff(const double* a, const double* b, int64_t n,
                              unsigned long long* acc_bits, hipStream_t s);

}  // namespace pic
