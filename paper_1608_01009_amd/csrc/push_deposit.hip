// Particle push and current deposition for one species (stages 2-4 of the
// PIC step of arXiv:1608.01009, Section 2: field interpolation, relativistic
// equations of motion, current deposition).
//
// One workgroup per supercell (Section 4.3 groups particles by supercells so
// that the grid data they touch stays close; here that data is staged in
// LDS):
//   1. the E/B values of the supercell plus an h-cell drift margin and the
//      one-node interpolation stencil are copied into an LDS tile,
//   2. each lane takes one particle at a time (SoA loads and stores are
//      coalesced because particles are sorted by supercell), gathers E/B
//      from the tile with cloud-in-cell weights, applies the Boris rotation,
//      advances the position, splits the move at cell planes
//      (Villasenor-Buneman) and accumulates the current of every segment
//      into an LDS J tile with ds_add_f64,
//   3. the J tile is added into the global J arrays with FP64 global atomics
//      (neighbouring tiles overlap by the halo, so the adds must be atomic).
// Particles that drifted further than the halo since the last re-sort take a
// global-memory path (gather from global E/B, global atomics for J).
//
// Gather, Boris and advance are evaluated in a fixed expression order (fused
// multiply-adds exactly where written, contraction off elsewhere, correctly
// rounded square roots and divisions), so positions and momenta are
// reproducible bit for bit by any IEEE FP64 evaluation of the same
// expressions.
#include "pic_device.h"
#include "pic_internal.h"

namespace pic {
namespace {

// 8 waves per workgroup; with two workgroups per CU (LDS) and at most 128
// VGPRs this keeps 4 waves on every SIMD.
constexpr int kBlock = 512;

// i mod n for i in [-n, 2n)
__device__ __forceinline__ int near_wrap(int i, int n) {
    i = i < 0 ? i + n : i;
    return i >= n ? i - n : i;
}

// Global linear index of tile node (tx, ty, tz) with tile origin org: the
// coordinates lie in [-n, 2n) when every n_d >= h + 2 (uniform flag `near`),
// otherwise they are reduced with a full modulo.
__device__ __forceinline__ int tile_node_index(const int org[3], int tx, int ty, int tz, int nx,
                                               int ny, int nz, bool near) {
    if (near)
        return near_wrap(org[0] + tx, nx) +
               nx * (near_wrap(org[1] + ty, ny) + ny * near_wrap(org[2] + tz, nz));
    return wrapi(org[0] + tx, nx) + nx * (wrapi(org[1] + ty, ny) + ny * wrapi(org[2] + tz, nz));
}

// Workgroups are dispatched round-robin over the 8 XCDs of the MI355X.  Map
// them so that each XCD receives a contiguous range of supercells: the
// overlapping halos of neighbouring tiles are then read and atomically
// updated through the same L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    if ((nb & 7) != 0) return b;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

struct PDArgs {
    Geom g;
    SpeciesC sp;
    Parts src;              // read: particle i of the new order at perm[i] (or i)
    Parts dst;              // written: particle i at i
    const unsigned* perm;   // nullptr: identity
    unsigned* keys;         // nullptr: no sort keys wanted
    const int* sc_off;
    const double* EB[6];
    double* J[3];
    unsigned* err;
    unsigned long long* nfar;
    int* far_q;          // indices of particles outside their supercell's tile
    unsigned* far_n;     // queue length for this launch
    unsigned* far_n_next;  // queue length of the next launch (cleared by far_kernel)
    DetJ det;              // deterministic mode: integer accumulators (hi[0] == nullptr: off)
};

// Arguments of NSP species pushed by one launch over one tile load per
// supercell (geometry, fields, J, error word and det shared: those of s[0]).
template <int NSP>
struct PDMulti {
    PDArgs s[NSP];
};

// Villasenor-Buneman current of one straight segment a -> b inside one cell,
// in cell-local coordinates (a, b in [0, 1]^3, both computed exactly from
// the positions).  J_d receives at the four d-directed edges of the cell
// jc_d dl_d W with W = w_p w_r +- dl_p dl_r / 12 (w at the segment midpoint,
// 1 - m or m per edge, p < r the transverse axes); the cross term
// jc_d dl_d dl_p dl_r / 12 is the same triple product dl_x dl_y dl_z for all
// three components.  emit(j, v) receives contribution j = 4 d + 2 bp + br
// (bp, br: the edge's offset along p and r).  J is summed by atomics in any
// order, so only the value of each contribution, not its rounding, is fixed.
template <class Emit>
__device__ __forceinline__ void vb_cell(const double a[3], const double b[3], const double jc[3],
                                        const Emit& emit) {
    double dl[3], m[3], w[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        dl[d] = b[d] - a[d];
        m[d] = 0.5 * (a[d] + b[d]);
        w[d] = 1.0 - m[d];
    }
    const double P = (dl[0] * dl[1]) * (dl[2] * (1.0 / 12.0));
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int p = d == 0 ? 1 : 0;
        const int r = d == 2 ? 1 : 2;
        const double f = jc[d] * dl[d];
        const double A = f * w[p], B = f * m[p], X = jc[d] * P;
        emit(4 * d + 0, __fma_rn(A, w[r], X));
        emit(4 * d + 1, __fma_rn(A, m[r], -X));
        emit(4 * d + 2, __fma_rn(B, w[r], -X));
        emit(4 * d + 3, __fma_rn(B, m[r], X));
        __builtin_amdgcn_sched_barrier(0);
    }
}

// One straight segment A->B inside the cell with integer corner `cell`:
// `sink(d, i, j, k, v)` adds v to J_d at the edge whose integer corner is
// lattice node (i, j, k) (unwrapped).
template <class Sink>
__device__ __forceinline__ void vb_segment(const double A[3], const double B[3],
                                           const int cell[3], const double jc[3],
                                           const Sink& sink) {
#pragma clang fp contract(off)
    double a[3], b[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        a[d] = A[d] - (double)cell[d];
        b[d] = B[d] - (double)cell[d];
    }
    vb_cell(a, b, jc, [&](int j, double v) {
        const int d = j >> 2, bp = (j >> 1) & 1, br = j & 1;
        const int p = d == 0 ? 1 : 0;
        const int r = d == 2 ? 1 : 2;
        int o[3] = {0, 0, 0};
        o[p] = bp;
        o[r] = br;
        sink(d, cell[0] + o[0], cell[1] + o[1], cell[2] + o[2], v);
    });
}

// Sort key of a stored (wrapped) position: supercell * S^3 + cell in
// supercell, both x-fastest.
template <int S>
__device__ __forceinline__ unsigned sort_key(const Geom& g, const double x[3]) {
    int c[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) c[d] = (int)floor(x[d]);
    const int sc = c[0] / S + g.ns[0] * (c[1] / S + g.ns[1] * (c[2] / S));
    const int loc = c[0] % S + S * (c[1] % S + S * (c[2] % S));
    return (unsigned)(sc * S * S * S + loc);
}

__device__ __forceinline__ unsigned sort_key_rt(const Geom& g, const double x[3]) {
    const int S = g.S;
    int c[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) c[d] = (int)floor(x[d]);
    const int sc = c[0] / S + g.ns[0] * (c[1] / S + g.ns[1] * (c[2] / S));
    const int loc = c[0] % S + S * (c[1] % S + S * (c[2] % S));
    return (unsigned)(sc * S * S * S + loc);
}

// Split x0 -> x1 at the cell planes it crosses, in order of crossing time
// (ties: x, y, z), and deposit every segment.  Each junction point is
// x0 + t (x1 - x0) with its crossing coordinate set to the plane exactly.
// The segment loop is kept rolled (the pending crossings rotate through three
// registers) so that this rare path needs few registers.
template <class Sink>
__device__ __forceinline__ void vb_move(const double x0[3], const double x1[3], const int c0[3],
                                        const int c1[3], const double jc[3], const Sink& sink) {
#pragma clang fp contract(off)
    double dv[3], pl[3], t[3];
    int dm[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        dv[d] = x1[d] - x0[d];
        const int p = c0[d] > c1[d] ? c0[d] : c1[d];
        pl[d] = (double)p;
        t[d] = (c1[d] != c0[d]) ? (pl[d] - x0[d]) / dv[d] : __builtin_huge_val();
        dm[d] = d;
    }
    int left = (c1[0] != c0[0]) + (c1[1] != c0[1]) + (c1[2] != c0[2]);
    cswap(t[0], dm[0], t[1], dm[1]);
    cswap(t[1], dm[1], t[2], dm[2]);
    cswap(t[0], dm[0], t[1], dm[1]);
    double A[3] = {x0[0], x0[1], x0[2]};
    int cell[3] = {c0[0], c0[1], c0[2]};
#pragma unroll 1
    for (;;) {
        double B[3];
#pragma unroll
        for (int d = 0; d < 3; ++d)
            B[d] = (left == 0) ? x1[d] : ((dm[0] == d) ? pl[d] : x0[d] + t[0] * dv[d]);
        vb_segment(A, B, cell, jc, sink);
        if (left == 0) break;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            A[d] = B[d];
            if (dm[0] == d) cell[d] = c1[d];
        }
        t[0] = t[1];
        dm[0] = dm[1];
        t[1] = t[2];
        dm[1] = dm[2];
        --left;
    }
}

// Gather of the six components given a loader ld(comp, ix, iy, iz, a, b, c)
// where (ix, iy, iz) is the lower stencil corner in the loader's frame.
template <class Ld>
__device__ __forceinline__ void gather6(const Stencil& st, const int off[3], const Ld& ld,
                                        double E[3], double Bf[3]) {
    // Yee stagger per component: Ex (h,0,0) Ey (0,h,0) Ez (0,0,h)
    //                            Bx (0,h,h) By (h,0,h) Bz (h,h,0)
    const int ix0 = st.i0[0] + off[0], iy0 = st.i0[1] + off[1], iz0 = st.i0[2] + off[2];
    const int ixh = st.ih[0] + off[0], iyh = st.ih[1] + off[1], izh = st.ih[2] + off[2];
    E[0] = cic8([&](int a, int b, int c) { return ld(0, ixh, iy0, iz0, a, b, c); },
                st.fh[0], st.f0[1], st.f0[2]);
    E[1] = cic8([&](int a, int b, int c) { return ld(1, ix0, iyh, iz0, a, b, c); },
                st.f0[0], st.fh[1], st.f0[2]);
    E[2] = cic8([&](int a, int b, int c) { return ld(2, ix0, iy0, izh, a, b, c); },
                st.f0[0], st.f0[1], st.fh[2]);
    Bf[0] = cic8([&](int a, int b, int c) { return ld(3, ix0, iyh, izh, a, b, c); },
                 st.f0[0], st.fh[1], st.fh[2]);
    Bf[1] = cic8([&](int a, int b, int c) { return ld(4, ixh, iy0, izh, a, b, c); },
                 st.fh[0], st.f0[1], st.fh[2]);
    Bf[2] = cic8([&](int a, int b, int c) { return ld(5, ixh, iyh, iz0, a, b, c); },
                 st.fh[0], st.fh[1], st.f0[2]);
}

// Tile gather of the six components.  Component k+1's eight values are
// loaded before component k is interpolated, so LDS latency overlaps the FMA
// chain with two components (32 VGPRs) in flight.  Same nested-lerp order as
// cic8: v[a + 2 b + 4 c] = F(a, b, c), x first, then y, then z.
struct Oct {
    double v[8];
};

template <int PY, int PZ>
__device__ __forceinline__ Oct ld_oct(const double* eb, int base) {
    // One address register per component (hiding the index from constant
    // folding keeps the component offset out of the loads, which then take
    // immediate offsets).  The loads are volatile so that they stay eight
    // single ds_read_b64: for the scattered addresses of a round of
    // particles, pairing them into ds_read2_b64 costs more LDS cycles than
    // the two single reads.
    asm volatile("" : "+v"(base));
    typedef __attribute__((address_space(3))) const volatile double lds_double;
    const lds_double* p = (const lds_double*)(eb + base);
    Oct o;
    o.v[0] = p[0];
    o.v[1] = p[1];
    o.v[2] = p[PY];
    o.v[3] = p[PY + 1];
    o.v[4] = p[PZ];
    o.v[5] = p[PZ + 1];
    o.v[6] = p[PZ + PY];
    o.v[7] = p[PZ + PY + 1];
    return o;
}

__device__ __forceinline__ double interp_oct(const Oct& o, double fx, double fy, double fz) {
#pragma clang fp contract(off)
    const double q00 = __fma_rn(fx, o.v[1] - o.v[0], o.v[0]);
    const double q10 = __fma_rn(fx, o.v[3] - o.v[2], o.v[2]);
    const double q01 = __fma_rn(fx, o.v[5] - o.v[4], o.v[4]);
    const double q11 = __fma_rn(fx, o.v[7] - o.v[6], o.v[6]);
    const double r0 = __fma_rn(fy, q10 - q00, q00);
    const double r1 = __fma_rn(fy, q11 - q01, q01);
    return __fma_rn(fz, r1 - r0, r0);
}

// The same from a tile of x-pairs (value, difference to x + 1): four 16-byte
// reads per component, and the x lerps take the stored difference.
typedef double vd2 __attribute__((ext_vector_type(2)));
struct Quad {
    vd2 p[4];
};

template <int PY, int PZ>
__device__ __forceinline__ Quad ld_quad(const double* eb, int base) {
    asm volatile("" : "+v"(base));
    typedef __attribute__((address_space(3))) const volatile vd2 lds_vd2;
    const lds_vd2* p = (const lds_vd2*)(eb + base);
    Quad o;
    o.p[0] = p[0];
    o.p[1] = p[PY / 2];
    o.p[2] = p[PZ / 2];
    o.p[3] = p[(PZ + PY) / 2];
    return o;
}

__device__ __forceinline__ double interp_quad(const Quad& o, double fx, double fy, double fz) {
#pragma clang fp contract(off)
    const double q00 = __fma_rn(fx, o.p[0].y, o.p[0].x);
    const double q10 = __fma_rn(fx, o.p[1].y, o.p[1].x);
    const double q01 = __fma_rn(fx, o.p[2].y, o.p[2].x);
    const double q11 = __fma_rn(fx, o.p[3].y, o.p[3].x);
    const double r0 = __fma_rn(fy, q10 - q00, q00);
    const double r1 = __fma_rn(fy, q11 - q01, q01);
    return __fma_rn(fz, r1 - r0, r0);
}

template <int PY, int PZ, int CS>
__device__ __forceinline__ void gather_tile_pairs(const double* eb, const Stencil& st,
                                                  const int off[3], double E[3], double Bf[3]) {
    const int x0 = 2 * (st.i0[0] + off[0]), y0 = st.i0[1] + off[1], z0 = st.i0[2] + off[2];
    const int xh = 2 * (st.ih[0] + off[0]), yh = st.ih[1] + off[1], zh = st.ih[2] + off[2];
    Quad a = ld_quad<PY, PZ>(eb, 0 * CS + xh + PY * y0 + PZ * z0);
    Quad b = ld_quad<PY, PZ>(eb, 1 * CS + x0 + PY * yh + PZ * z0);
    E[0] = interp_quad(a, st.fh[0], st.f0[1], st.f0[2]);
    a = ld_quad<PY, PZ>(eb, 2 * CS + x0 + PY * y0 + PZ * zh);
    E[1] = interp_quad(b, st.f0[0], st.fh[1], st.f0[2]);
    b = ld_quad<PY, PZ>(eb, 3 * CS + x0 + PY * yh + PZ * zh);
    E[2] = interp_quad(a, st.f0[0], st.f0[1], st.fh[2]);
    a = ld_quad<PY, PZ>(eb, 4 * CS + xh + PY * y0 + PZ * zh);
    Bf[0] = interp_quad(b, st.f0[0], st.fh[1], st.fh[2]);
    b = ld_quad<PY, PZ>(eb, 5 * CS + xh + PY * yh + PZ * z0);
    Bf[1] = interp_quad(a, st.fh[0], st.f0[1], st.fh[2]);
    Bf[2] = interp_quad(b, st.fh[0], st.fh[1], st.f0[2]);
}

template <class EL>
__device__ __forceinline__ void gather_tile(const double* eb, const Stencil& st, const int off[3],
                                            double E[3], double Bf[3]) {
    constexpr int PY = EL::PY, PZ = EL::PZ, CS = EL::CS;
    if constexpr (EL::kPair) {
        gather_tile_pairs<PY, PZ, CS>(eb, st, off, E, Bf);
        return;
    }
    const int x0 = st.i0[0] + off[0], y0 = st.i0[1] + off[1], z0 = st.i0[2] + off[2];
    const int xh = st.ih[0] + off[0], yh = st.ih[1] + off[1], zh = st.ih[2] + off[2];
    // Yee stagger per component: Ex (h,0,0) Ey (0,h,0) Ez (0,0,h)
    //                            Bx (0,h,h) By (h,0,h) Bz (h,h,0)
    Oct a = ld_oct<PY, PZ>(eb, 0 * CS + xh + PY * y0 + PZ * z0);
    Oct b = ld_oct<PY, PZ>(eb, 1 * CS + x0 + PY * yh + PZ * z0);
    E[0] = interp_oct(a, st.fh[0], st.f0[1], st.f0[2]);
    a = ld_oct<PY, PZ>(eb, 2 * CS + x0 + PY * y0 + PZ * zh);
    E[1] = interp_oct(b, st.f0[0], st.fh[1], st.f0[2]);
    b = ld_oct<PY, PZ>(eb, 3 * CS + x0 + PY * yh + PZ * zh);
    E[2] = interp_oct(a, st.f0[0], st.f0[1], st.fh[2]);
    a = ld_oct<PY, PZ>(eb, 4 * CS + xh + PY * y0 + PZ * zh);
    Bf[0] = interp_oct(b, st.f0[0], st.fh[1], st.fh[2]);
    b = ld_oct<PY, PZ>(eb, 5 * CS + xh + PY * yh + PZ * z0);
    Bf[1] = interp_oct(a, st.fh[0], st.f0[1], st.fh[2]);
    Bf[2] = interp_oct(b, st.fh[0], st.fh[1], st.f0[2]);
}

__device__ __forceinline__ bool finite3(double a, double b, double c) {
    return isfinite(a) && isfinite(b) && isfinite(c);
}

// The twelve J contributions of one segment that stays inside one cell,
// ordered (d, bp, br) with d the J component and (bp, br) the offsets along
// its two transverse axes in increasing axis order; add(j, v) receives them
// one component at a time.
template <class Add>
__device__ __forceinline__ void vb_single(const double x0[3], const double x1[3], const int c[3],
                                          const double jc[3], const Add& add) {
#pragma clang fp contract(off)
    double a[3], b[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        a[d] = x0[d] - (double)c[d];
        b[d] = x1[d] - (double)c[d];
    }
    vb_cell(a, b, jc, add);
}

// Layout of the E/B tile in LDS.  PAIR: x-pairs; for node (tx, ty, tz) of
// component c with tx < T - 1, the value at c * CS + 2 tx + PY * ty + PZ * tz
// and, beside it, the difference to the next node in x (what the first lerp
// of the interpolation subtracts, formed once per node instead of once per
// particle; the same FP64 subtraction, so the result is unchanged): one
// 16-byte read per pair.  Otherwise node (tx, ty, tz) at c * CS + tx + PY * ty
// + PZ * tz.  For S = 4 the plane pitch is padded by 4 doubles, which spreads
// the stencils of the lanes of a round (two z-layers of the supercell per half
// wave, each lane shifted by the component's stagger) over more LDS banks.
template <int S, int H, bool PAIR>
struct EBLayout {
    static constexpr int T = S + 2 * H + 2;
    static constexpr bool kPair = PAIR;
    static constexpr int PY = PAIR ? 2 * (T - 1) : T;
    static constexpr int PZ = (S == 4) ? PY * T + 4 : PY * T;
    static constexpr int CS = PZ * T;  // doubles per component
};

// Layout of the J tile in LDS: node (tx, ty, tz) of component d lives at
// d * JC + tx + PY * ty + PZ * tz.  For S = 4 the pitches are padded so that
// the 32 cells of a half wave (one round covers the 64 cells of the
// supercell) fall on 32 distinct bank pairs for every one of the twelve
// contributions, which keeps the FP64 LDS atomics free of bank conflicts.
template <int S, int H>
struct JLayout {
    static constexpr int TJ = S + 2 * H + 3;
    static constexpr int PY = (S == 4 && H == 1) ? 12 : TJ;
    static constexpr int PZ = (S == 4 && H == 1) ? 112 : TJ * TJ;
    static constexpr int JC = PZ * (TJ - 1) + PY * (TJ - 1) + TJ;  // doubles per component
};

// LDS offset (relative to the node of the cell) of contribution j of
// vb_single: j = 4 d + 2 bp + br.
template <int PY, int PZ, int JC>
__device__ __forceinline__ constexpr int jt_off(int j) {
    const int d = j >> 2, bp = (j >> 1) & 1, br = j & 1;
    // d = 0: (p, r) = (y, z); d = 1: (x, z); d = 2: (x, y)
    const int sp = (d == 0) ? PY : 1;
    const int sr = (d == 2) ? PY : PZ;
    return d * JC + bp * sp + br * sr;
}

// GATHER: particle i of this step is read from src at perm[i] (the step after
// a re-sort), otherwise at i.
// DET: the J tile and the flush use the exact integer split (DetJ).
// ABS: absorbing x boundaries: lattice points outside 0 <= x < n0 read zero
// and receive no current; a particle whose move ends outside 0 <= x < n0 - 1
// is stored with x = -1 (removed) and later skipped.
// NSP: species pushed one after the other over the same E/B tile and into the
// same J tile (one tile load and one flush per supercell for all of them).
template <int S, int H, bool GATHER, bool DET, bool ABS, int NSP>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4)))
push_deposit_kernel(const PDMulti<NSP> m) {
    const PDArgs& a = m.s[0];   // shared: geometry, fields, J, det, error word
    // x-pairs for one species without DET: with DET's larger J tile they would
    // leave one workgroup per CU, and the two-species kernels spill with them
    using EL = EBLayout<S, H, !DET && NSP == 1>;
    constexpr int T = EL::T;           // E/B tile edge in nodes
    constexpr int T2 = T * T, T3 = T2 * T;
    using JL = JLayout<S, H>;
    constexpr int TJ = JL::TJ;         // J tile edge in nodes
    constexpr int PY = JL::PY, PZ = JL::PZ, JC = JL::JC;
    constexpr int kWaves = kBlock / 64;
    constexpr int QCAP = 28;           // queued cell-crossing particles per wave
    __shared__ __attribute__((aligned(16))) double eb[6 * EL::CS];
    // J tile: FP64 sums, or (DET) 64-bit hi sums followed by 32-bit lo sums
    constexpr int JT_BYTES = DET ? 3 * JC * 12 : 3 * JC * 8;
    __shared__ __attribute__((aligned(16))) unsigned char jraw[JT_BYTES];
    double* const jt = (double*)jraw;
    unsigned long long* const jth = (unsigned long long*)jraw;
    int* const jtl = (int*)(jraw + 3 * JC * 8);
    auto jadd = [&](int idx, double v) {
        if (DET) {
            unsigned long long h;
            int l;
            det_split(v, a.det.scale, h, l);
            atomicAdd(&jth[idx], h);
            atomicAdd(&jtl[idx], l);
        } else {
            atomicAdd(&jt[idx], v);
        }
    };
    __shared__ double qb[kWaves][6][QCAP];

    const int sc = xcd_block(blockIdx.x, gridDim.x);
    const Geom& g = a.g;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const int sx = sc % g.ns[0];
    const int syz = sc / g.ns[0];
    const int sy = syz % g.ns[1], sz = syz / g.ns[1];
    const int base[3] = {sx * S, sy * S, sz * S};          // first cell of the supercell
    const int org[3] = {base[0] - H - 1, base[1] - H - 1, base[2] - H - 1};  // tile origin
    const bool near = nx >= H + 2 && ny >= H + 2 && nz >= H + 2;
    // E/B tile values of this thread's nodes: one wrapped global index per
    // node, shared by the six components (tile coordinates lie within one
    // period of [0, n)).  SPEC: one species on periodic boundaries, where
    // supercells are rarely empty: the tile loads go out before the particle
    // ranges arrive, so that the two latencies overlap.
    constexpr bool SPEC = NSP == 1 && !ABS;
    constexpr int TN = (T3 + kBlock - 1) / kBlock;
    double tv[TN][6];
    auto tile_loads = [&]() {
#pragma unroll
        for (int i = 0; i < TN; ++i) {
            const int r = (int)threadIdx.x + i * kBlock;
            if (r < T3) {
                const int tz = r / T2, ty = (r / T) % T, tx = r % T;
                const int gi = tile_node_index(org, tx, ty, tz, nx, ny, nz, near);
                const bool outside = ABS && (org[0] + tx < 0 || org[0] + tx >= nx);
#pragma unroll
                for (int c = 0; c < 6; ++c) tv[i][c] = outside ? 0.0 : a.EB[c][gi];
            }
        }
    };
    if (SPEC) tile_loads();
    {
        // empty supercell: uniform exit before any barrier
        bool any = false, over = false;
#pragma unroll
        for (int si = 0; si < NSP; ++si) {
            const int q0 = m.s[si].sc_off[sc], q1 = m.s[si].sc_off[sc + 1];
            any = any || q0 < q1;
            over = over || (DET && q1 - q0 > kDetMaxPerSupercell);
        }
        if (!any) return;
        if (over) {
            if (threadIdx.x == 0) atomicOr(a.err, ERR_DETCAP);
            return;
        }
    }

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const unsigned long long lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    // software pipeline: the next particle's state is loaded one iteration
    // ahead; the first particle's loads and the tile loads are in flight
    // together (with more than one species, or absorbing x, the particle
    // loads go first; otherwise the tile loads, see SPEC above)
    double nxt[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    // Particle arrays are addressed with 32-bit byte offsets from the scalar
    // base of each array (arrays are below 4 GiB: capacity < 2^29), so the
    // six loads and six stores of a particle share one offset register.
    auto ld6 = [&](const PDArgs& as, unsigned j, double o[6]) {
        const unsigned b = j * 8u;
        o[0] = *(const double*)((const char*)as.src.x + b);
        o[1] = *(const double*)((const char*)as.src.y + b);
        o[2] = *(const double*)((const char*)as.src.z + b);
        o[3] = *(const double*)((const char*)as.src.ux + b);
        o[4] = *(const double*)((const char*)as.src.uy + b);
        o[5] = *(const double*)((const char*)as.src.uz + b);
    };
    // GATHER: the re-sort order is read two iterations ahead of the data it
    // addresses, so that issuing the next particle's loads never waits on a
    // just-issued order load (the vector memory counter completes in issue
    // order, and such a wait would also wait for this iteration's stores).
    unsigned pj = 0;
    auto first_loads = [&](const PDArgs& as) {
        const int q0 = as.sc_off[sc], q1 = as.sc_off[sc + 1];
        const int ip = q0 + (int)threadIdx.x;
        if (GATHER) {
            if (ip < q1) ld6(as, as.perm[ip], nxt);
            if (ip + kBlock < q1) pj = as.perm[ip + kBlock];
        } else {
            // every lane loads (past the end: the spare slot), so that the
            // count of loads in flight is known where the tile values are
            // consumed, and that wait leaves these loads in flight
            ld6(as, ip < q1 ? (unsigned)ip : as.src.spare, nxt);
        }
    };
    first_loads(m.s[0]);
    if (!SPEC) tile_loads();
#pragma unroll
    for (int i = 0; i < TN; ++i) {
        const int r = (int)threadIdx.x + i * kBlock;
        if (r < T3) {
            const int tz = r / T2, ty = (r / T) % T, tx = r % T;
            // x-pairs: the values first (the last node of a row in the
            // difference slot of the pair before it), then the differences
            const int lx = !EL::kPair ? tx : (tx < T - 1 ? 2 * tx : 2 * T - 3);
            const int li = lx + EL::PY * ty + EL::PZ * tz;
#pragma unroll
            for (int c = 0; c < 6; ++c) eb[c * EL::CS + li] = tv[i][c];
        }
    }
    for (int t = threadIdx.x; t < JT_BYTES / 4; t += kBlock) ((int*)jraw)[t] = 0;
    __syncthreads();
    if constexpr (EL::kPair) {
#pragma unroll
        for (int i = 0; i < TN; ++i) {
            const int r = (int)threadIdx.x + i * kBlock;
            const int tz = r / T2, ty = (r / T) % T, tx = r % T;
            if (r < T3 && tx < T - 1) {
                const int li = 2 * tx + EL::PY * ty + EL::PZ * tz;
                const int ln = tx < T - 2 ? li + 2 : li + 1;
#pragma unroll
                for (int c = 0; c < 6; ++c)
                    eb[c * EL::CS + li + 1] = eb[c * EL::CS + ln] - tv[i][c];
            }
        }
        __syncthreads();
    }

    const double L[3] = {(double)nx, (double)ny, (double)nz};
    const int nn[3] = {nx, ny, nz};

    // relative cell of c0 inside the tile window [-H, S+H), periodic
    auto relcell = [&](const int c0[3], int rel[3]) {
        bool in = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int r = c0[d] - base[d];
            if (r >= S + H)
                r -= nn[d];
            else if (r < -H)
                r += nn[d];
            rel[d] = r;
            in = in && (r >= -H) && (r < S + H);
        }
        return in;
    };
#pragma unroll 1
    for (int si = 0; si < NSP; ++si) {
    const PDArgs& a = m.s[si];
    const int p0 = a.sc_off[sc], p1 = a.sc_off[sc + 1];
    if (si > 0) first_loads(a);
    // deposit of a general move (any number of plane crossings) into the tile
    auto deposit_tile = [&](const double x0[3], const double x1[3]) {
        int c0[3], c1[3], rel[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            c0[d] = (int)floor(x0[d]);
            c1[d] = (int)floor(x1[d]);
        }
        relcell(c0, rel);
        const int jo0 = rel[0] + H + 1 - c0[0], jo1 = rel[1] + H + 1 - c0[1],
                  jo2 = rel[2] + H + 1 - c0[2];
        vb_move(x0, x1, c0, c1, a.sp.jc, [&](int d, int i, int j, int k, double v) {
            jadd(d * JC + (i + jo0) + PY * (j + jo1) + PZ * (k + jo2), v);
        });
    };
    // queued crossers of this wave: one per lane, then the queue is empty
    auto drain = [&](int cnt) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < cnt) {
            const double q0[3] = {qb[wv][0][lane], qb[wv][1][lane], qb[wv][2][lane]};
            const double q1[3] = {qb[wv][3][lane], qb[wv][4][lane], qb[wv][5][lane]};
            deposit_tile(q0, q1);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };

    int qcount = 0;  // wave-uniform
    for (int pb = p0; pb < p1; pb += kBlock) {
        const int ip = pb + (int)threadIdx.x;
        const bool valid = ip < p1;
        double x0[3] = {nxt[0], nxt[1], nxt[2]};
        double u[3] = {nxt[3], nxt[4], nxt[5]};
        {
            const int in = ip + kBlock;
            if (in < p1) ld6(a, GATHER ? pj : (unsigned)in, nxt);
            if (GATHER && in + kBlock < p1) pj = a.perm[in + kBlock];
        }
        bool crosser = false, far = false;
        double x1[3] = {0.0, 0.0, 0.0};
        // Every lane stores; lanes without a pushed particle (past the end
        // of the supercell, far movers, whose slot far_kernel rewrites, and
        // non-finite states) store to the spare slot.  The stores then sit on
        // every path of the loop body, so the wait for the next particle's
        // prefetched loads does not also wait for this particle's stores.
        unsigned o = a.dst.spare;
        double xw[3] = {0.0, 0.0, 0.0};
        // removed particles (absorbing x) keep their slot untouched; a
        // re-sort that follows sorts them after every cell
        const bool dead = ABS && valid && x0[0] < 0.0;
        if (dead && a.keys) a.keys[ip] = (unsigned)g.ncell;
        if (valid && !dead) {
            // stored positions lie in [0, L) (this also rejects NaN); a
            // non-finite momentum shows up in the pushed state checked below
            bool ok = (x0[0] >= 0.0 && x0[0] < L[0]) && (x0[1] >= 0.0 && x0[1] < L[1]) &&
                      (x0[2] >= 0.0 && x0[2] < L[2]);
            double fl[3];
            int c0[3], rel[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                fl[d] = ok ? floor(x0[d]) : 0.0;
                c0[d] = (int)fl[d];
            }
            const bool inside = ok && relcell(c0, rel);
            far = ok && !inside;
            if (inside) {
                Stencil st;
                make_stencil(x0, fl, st);
                double E[3], Bf[3];
                int off[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) off[d] = rel[d] + H + 1 - c0[d];
                gather_tile<EL>(eb, st, off, E, Bf);
                boris_advance(a.sp, g, E, Bf, u, x0, x1);
                ok = finite3(u[0], u[1], u[2]) && finite3(x1[0], x1[1], x1[2]);
            }
            if (!ok) {
                atomicOr(a.err, ERR_NONFINITE);
            } else if (inside) {
                int c1[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) c1[d] = (int)floor(x1[d]);
                if (c1[0] == c0[0] && c1[1] == c0[1] && c1[2] == c0[2]) {
                    // single-cell move: twelve LDS atomic adds; within a round
                    // of the stored order the lanes of a wave sit in distinct
                    // cells
                    const int key =
                        (rel[0] + H + 1) + PY * (rel[1] + H + 1) + PZ * (rel[2] + H + 1);
                    vb_single(x0, x1, c0, a.sp.jc, [&](int j, double v) {
                        jadd(key + jt_off<PY, PZ, JC>(j), v);
                    });
                } else {
                    crosser = true;
                }
                // positions are stored wrapped into [0, n)
#pragma unroll
                for (int d = 0; d < 3; ++d) xw[d] = wrap_coord(x1[d], L[d]);
                if (ABS && !(x1[0] >= 0.0 && x1[0] < L[0] - 1.0)) xw[0] = -1.0;   // removed
                o = (unsigned)ip;
            }
        }
        {
            const unsigned b = o * 8u;
            *(double*)((char*)a.dst.x + b) = xw[0];
            *(double*)((char*)a.dst.y + b) = xw[1];
            *(double*)((char*)a.dst.z + b) = xw[2];
            *(double*)((char*)a.dst.ux + b) = u[0];
            *(double*)((char*)a.dst.uy + b) = u[1];
            *(double*)((char*)a.dst.uz + b) = u[2];
            if (a.keys && o != a.dst.spare)
                a.keys[o] = (ABS && xw[0] < 0.0) ? (unsigned)g.ncell : sort_key<S>(g, xw);
        }

        // Far movers (outside the tile window) are left untouched here and
        // queued for far_kernel, which gathers and deposits through global
        // memory.
        {
            const unsigned long long fm = __ballot(far);
            if (fm) {
                const int lead = __ffsll((long long)fm) - 1;
                unsigned base = 0;
                if (lane == lead) base = atomicAdd(a.far_n, (unsigned)__popcll(fm));
                base = (unsigned)__builtin_amdgcn_readlane((int)base, lead);
                if (far) a.far_q[base + (unsigned)__popcll(fm & lt_mask)] = ip;
            }
        }

        // Cell-crossing moves: queued per wave, deposited one per lane.
        {
            const unsigned long long cm = __ballot(crosser);
            const int nnew = __popcll(cm);
            if (nnew > QCAP) {
                if (crosser) deposit_tile(x0, x1);
            } else if (nnew > 0) {
                if (qcount + nnew > QCAP) {
                    drain(qcount);
                    qcount = 0;
                }
                if (crosser) {
                    const int slot = qcount + __popcll(cm & lt_mask);
                    qb[wv][0][slot] = x0[0];
                    qb[wv][1][slot] = x0[1];
                    qb[wv][2][slot] = x0[2];
                    qb[wv][3][slot] = x1[0];
                    qb[wv][4][slot] = x1[1];
                    qb[wv][5][slot] = x1[2];
                }
                qcount += nnew;
            }
        }
    }
    if (qcount > 0) drain(qcount);
    }  // species
    __syncthreads();

    constexpr int TJ2 = TJ * TJ, TJ3 = TJ2 * TJ;
    for (int r = threadIdx.x; r < TJ3; r += kBlock) {
        const int tz = r / TJ2, ty = (r / TJ) % TJ, tx = r % TJ;
        const int li = tx + PY * ty + PZ * tz;
        if (ABS && (org[0] + tx < 0 || org[0] + tx >= nx)) continue;   // outside the box
        if (DET) {
            const unsigned long long h[3] = {jth[li], jth[JC + li], jth[2 * JC + li]};
            const int l[3] = {jtl[li], jtl[JC + li], jtl[2 * JC + li]};
            if ((h[0] | h[1] | h[2]) != 0ull || (l[0] | l[1] | l[2]) != 0) {
                const int gi = tile_node_index(org, tx, ty, tz, nx, ny, nz, near);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if (h[c] != 0ull) atomicAdd(&a.det.hi[c][gi], h[c]);
                    if (l[c] != 0)
                        atomicAdd((unsigned long long*)&a.det.lo[c][gi],
                                  (unsigned long long)(long long)l[c]);
                }
            }
        } else {
            const double v[3] = {jt[li], jt[JC + li], jt[2 * JC + li]};
            if (v[0] != 0.0 || v[1] != 0.0 || v[2] != 0.0) {
                const int gi = tile_node_index(org, tx, ty, tz, nx, ny, nz, near);
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    if (v[c] != 0.0) unsafeAtomicAdd(&a.J[c][gi], v[c]);
            }
        }
    }
}

// Particles that drifted beyond the halo of their supercell's tile since the
// last re-sort: gather from the global E/B arrays, push, deposit with global
// FP64 atomics, wrap and store.  The queue was filled by push_deposit_kernel.
__global__ void __launch_bounds__(kBlock) far_kernel(const PDArgs a) {
    const unsigned n = *a.far_n;
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.far_n_next = 0u;
    const Geom& g = a.g;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const double L[3] = {(double)nx, (double)ny, (double)nz};
    unsigned long long cnt = 0;
    // queue entry i goes to workgroup i mod gridDim: a short queue (the usual
    // case) spreads one particle per workgroup over the CUs instead of
    // filling the waves of the first workgroup
    for (unsigned i = threadIdx.x * gridDim.x + blockIdx.x; i < n; i += gridDim.x * kBlock) {
        const int ip = a.far_q[i];
        const unsigned j = a.perm ? a.perm[ip] : (unsigned)ip;
        double x0[3] = {a.src.x[j], a.src.y[j], a.src.z[j]};
        double u[3] = {a.src.ux[j], a.src.uy[j], a.src.uz[j]};
        double fl[3];
        int c0[3], c1[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            fl[d] = floor(x0[d]);
            c0[d] = (int)fl[d];
        }
        Stencil st;
        make_stencil(x0, fl, st);
        double E[3], Bf[3], x1[3];
        const int off[3] = {0, 0, 0};
        gather6(st, off,
                [&](int comp, int ix, int iy, int iz, int da, int db, int dc) {
                    if (g.absorb_x && (ix + da < 0 || ix + da >= nx)) return 0.0;
                    return a.EB[comp][wrapi(ix + da, nx) +
                                      nx * (wrapi(iy + db, ny) + ny * wrapi(iz + dc, nz))];
                },
                E, Bf);
        boris_advance(a.sp, g, E, Bf, u, x0, x1);
        if (!(finite3(u[0], u[1], u[2]) && finite3(x1[0], x1[1], x1[2]))) {
            atomicOr(a.err, ERR_NONFINITE);
            continue;
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) c1[d] = (int)floor(x1[d]);
        vb_move(x0, x1, c0, c1, a.sp.jc, [&](int d, int i, int j, int k, double vv) {
            if (g.absorb_x && (i < 0 || i >= nx)) return;      // outside the box
            const int gi = wrapi(i, nx) + nx * (wrapi(j, ny) + ny * wrapi(k, nz));
            if (a.det.hi[0]) {
                unsigned long long h;
                int l;
                det_split(vv, a.det.scale, h, l);
                atomicAdd(&a.det.hi[d][gi], h);
                atomicAdd((unsigned long long*)&a.det.lo[d][gi], (unsigned long long)(long long)l);
            } else {
                unsafeAtomicAdd(&a.J[d][gi], vv);
            }
        });
        const bool removed = g.absorb_x && !(x1[0] >= 0.0 && x1[0] < L[0] - 1.0);
        const double xw[3] = {removed ? -1.0 : wrap_coord(x1[0], L[0]), wrap_coord(x1[1], L[1]),
                              wrap_coord(x1[2], L[2])};
        a.dst.x[ip] = xw[0];
        a.dst.y[ip] = xw[1];
        a.dst.z[ip] = xw[2];
        a.dst.ux[ip] = u[0];
        a.dst.uy[ip] = u[1];
        a.dst.uz[ip] = u[2];
        if (a.keys) a.keys[ip] = removed ? (unsigned)g.ncell : sort_key_rt(g, xw);
        cnt += 1;
    }
    if (cnt) atomicAdd(a.nfar, cnt);
}

// Absorbing x boundaries are compiled for these (S, h) pairs only.
template <int S, int H>
constexpr bool abs_supported() {
    return (S == 2 || S == 4) && (H == 1 || H == 2);
}

template <int S, int H>
hipError_t launch_sh(const PDArgs& args, hipStream_t s) {
    const bool det = args.det.hi[0] != nullptr;
    const PDMulti<1> m{{args}};
    if constexpr (abs_supported<S, H>()) {
        if (args.g.absorb_x) {
            if (det) return hipErrorInvalidValue;
            if (args.perm)
                hipLaunchKernelGGL((push_deposit_kernel<S, H, true, false, true, 1>),
                                   dim3(args.g.nsc), dim3(kBlock), 0, s, m);
            else
                hipLaunchKernelGGL((push_deposit_kernel<S, H, false, false, true, 1>),
                                   dim3(args.g.nsc), dim3(kBlock), 0, s, m);
            return hipGetLastError();
        }
    } else {
        if (args.g.absorb_x) return hipErrorInvalidValue;
    }
    if (args.perm && det)
        hipLaunchKernelGGL((push_deposit_kernel<S, H, true, true, false, 1>), dim3(args.g.nsc),
                           dim3(kBlock), 0, s, m);
    else if (args.perm)
        hipLaunchKernelGGL((push_deposit_kernel<S, H, true, false, false, 1>), dim3(args.g.nsc),
                           dim3(kBlock), 0, s, m);
    else if (det)
        hipLaunchKernelGGL((push_deposit_kernel<S, H, false, true, false, 1>), dim3(args.g.nsc),
                           dim3(kBlock), 0, s, m);
    else
        hipLaunchKernelGGL((push_deposit_kernel<S, H, false, false, false, 1>), dim3(args.g.nsc),
                           dim3(kBlock), 0, s, m);
    return hipGetLastError();
}

// Two species over one tile load (compiled where absorbing x is: S 2 or 4,
// h 1 or 2; not for the deterministic J).
template <int S, int H>
hipError_t launch_sh_pair(const PDArgs& a0, const PDArgs& a1, hipStream_t s) {
    if constexpr (abs_supported<S, H>()) {
        if (a0.det.hi[0] != nullptr || (a0.perm == nullptr) != (a1.perm == nullptr))
            return hipErrorInvalidValue;
        const PDMulti<2> m{{a0, a1}};
        const bool gather = a0.perm != nullptr;
        if (a0.g.absorb_x) {
            if (gather)
                hipLaunchKernelGGL((push_deposit_kernel<S, H, true, false, true, 2>),
                                   dim3(a0.g.nsc), dim3(kBlock), 0, s, m);
            else
                hipLaunchKernelGGL((push_deposit_kernel<S, H, false, false, true, 2>),
                                   dim3(a0.g.nsc), dim3(kBlock), 0, s, m);
        } else {
            if (gather)
                hipLaunchKernelGGL((push_deposit_kernel<S, H, true, false, false, 2>),
                                   dim3(a0.g.nsc), dim3(kBlock), 0, s, m);
            else
                hipLaunchKernelGGL((push_deposit_kernel<S, H, false, false, false, 2>),
                                   dim3(a0.g.nsc), dim3(kBlock), 0, s, m);
        }
        return hipGetLastError();
    } else {
        (void)a0;
        (void)a1;
        (void)s;
        return hipErrorInvalidValue;
    }
}

template <int S, int H>
constexpr int lds_bytes_sh(bool det) {
    return (6 * (det ? EBLayout<S, H, false>::CS : EBLayout<S, H, true>::CS) +
            (kBlock / 64) * 6 * 28) * (int)sizeof(double) +
           3 * JLayout<S, H>::JC * (det ? 12 : 8);
}

}  // namespace

// Supported (S, h) pairs (the LDS tiles of one workgroup must fit in the
// 160 KiB of a CU).
#define PIC_SH_TABLE(X) \
    X(1, 1) X(1, 2) X(2, 1) X(2, 2) X(3, 1) X(4, 1) X(4, 2) X(5, 1) X(6, 1)

bool push_deposit_supported(int S, int h) {
#define PIC_X(s_, h_) if (S == s_ && h == h_) return true;
    PIC_SH_TABLE(PIC_X)
#undef PIC_X
    return false;
}

int push_deposit_lds_bytes(const Geom& g, bool det) {
#define PIC_X(s_, h_) if (g.S == s_ && g.h == h_) return lds_bytes_sh<s_, h_>(det);
    PIC_SH_TABLE(PIC_X)
#undef PIC_X
    return -1;
}

namespace {

PDArgs make_args(const Geom& g, const SpeciesC& sp, const Parts& src, const Parts& dst,
                 const unsigned* perm, unsigned* keys, const int* sc_off, const Fields& f,
                 double* const J[3], unsigned* err, unsigned long long* nfar, int* far_q,
                 unsigned* far_n, unsigned* far_n_next, const DetJ& det) {
    PDArgs args;
    args.det = det;
    args.g = g;
    args.sp = sp;
    args.src = src;
    args.dst = dst;
    args.perm = perm;
    args.keys = keys;
    args.sc_off = sc_off;
    for (int c = 0; c < 3; ++c) {
        args.EB[c] = f.E[c];
        args.EB[3 + c] = f.B[c];
        args.J[c] = J[c];
    }
    args.err = err;
    args.nfar = nfar;
    args.far_q = far_q;
    args.far_n = far_n;
    args.far_n_next = far_n_next;
    return args;
}

}  // namespace

hipError_t launch_push_deposit(const Geom& g, const SpeciesC& sp, const Parts& src,
                               const Parts& dst, const unsigned* perm, unsigned* keys,
                               const int* sc_off, const Fields& f, double* const J[3],
                               unsigned* err, unsigned long long* nfar, int* far_q,
                               unsigned* far_n, unsigned* far_n_next, const DetJ& det,
                               hipStream_t s) {
    const PDArgs args = make_args(g, sp, src, dst, perm, keys, sc_off, f, J, err, nfar, far_q,
                                  far_n, far_n_next, det);
    if (g.nsc <= 0) return hipSuccess;
#define PIC_X(s_, h_) if (g.S == s_ && g.h == h_) return launch_sh<s_, h_>(args, s);
    PIC_SH_TABLE(PIC_X)
#undef PIC_X
    return hipErrorInvalidValue;
}

bool push_deposit_pair_supported(int S, int h, bool det) {
    return !det && (S == 2 || S == 4) && (h == 1 || h == 2);
}

hipError_t launch_push_deposit_pair(const Geom& g, const SpeciesC* sp, const Parts* src,
                                    const Parts* dst, const unsigned* const* perm,
                                    unsigned* const* keys, const int* const* sc_off,
                                    const Fields& f, double* const J[3], unsigned* err,
                                    unsigned long long* nfar, int* const* far_q,
                                    unsigned* const* far_n, unsigned* const* far_n_next,
                                    const DetJ& det, hipStream_t s) {
    const PDArgs a0 = make_args(g, sp[0], src[0], dst[0], perm[0], keys[0], sc_off[0], f, J,
                                err, nfar, far_q[0], far_n[0], far_n_next[0], det);
    const PDArgs a1 = make_args(g, sp[1], src[1], dst[1], perm[1], keys[1], sc_off[1], f, J,
                                err, nfar, far_q[1], far_n[1], far_n_next[1], det);
    if (g.nsc <= 0) return hipSuccess;
    if (g.S == 2 && g.h == 1) return launch_sh_pair<2, 1>(a0, a1, s);
    if (g.S == 2 && g.h == 2) return launch_sh_pair<2, 2>(a0, a1, s);
    if (g.S == 4 && g.h == 1) return launch_sh_pair<4, 1>(a0, a1, s);
    if (g.S == 4 && g.h == 2) return launch_sh_pair<4, 2>(a0, a1, s);
    return hipErrorInvalidValue;
}

namespace {

// The push's square root and division on arrays (the library's self-check),
// FP64 or (mixed-precision push) FP32.
template <class F>
__global__ void __launch_bounds__(256) sqrt_div_kernel(int64_t n, const F* x, const F* a,
                                                      const F* b, F* sq, F* dv) {
    for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        if constexpr (sizeof(F) == 8) {
            if (sq) sq[i] = sqrt_ge1(x[i]);
            if (dv) dv[i] = div_ge1(a[i], b[i]);
        } else {
            if (sq) sq[i] = sqrt_ge1_f32(x[i]);
            if (dv) dv[i] = div_ge1_f32(a[i], b[i]);
        }
    }
}

}  // namespace

hipError_t launch_sqrt_div(int64_t n, const double* x, const double* a, const double* b,
                           double* sq, double* dv, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(sqrt_div_kernel<double>, dim3((unsigned)nb), dim3(256), 0, s, n, x, a, b,
                       sq, dv);
    return hipGetLastError();
}

hipError_t launch_sqrt_div_f32(int64_t n, const float* x, const float* a, const float* b,
                               float* sq, float* dv, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(sqrt_div_kernel<float>, dim3((unsigned)nb), dim3(256), 0, s, n, x, a, b,
                       sq, dv);
    return hipGetLastError();
}

hipError_t launch_far_movers(const Geom& g, const SpeciesC& sp, const Parts& src,
                             const Parts& dst, const unsigned* perm, unsigned* keys,
                             const Fields& f, double* const J[3], unsigned* err,
                             unsigned long long* nfar, int* far_q, unsigned* far_n,
                             unsigned* far_n_next, const DetJ& det, hipStream_t s) {
    const PDArgs args = make_args(g, sp, src, dst, perm, keys, nullptr, f, J, err, nfar, far_q,
                                  far_n, far_n_next, det);
    hipLaunchKernelGGL(far_kernel, dim3(256), dim3(kBlock), 0, s, args);
    return hipGetLastError();
}

}  // namespace pic
