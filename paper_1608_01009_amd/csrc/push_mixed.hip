// Mixed-precision particle push and current deposition: the same stages and
// workgroup structure as push_deposit.hip (one workgroup per supercell, E/B
// and J tiles in LDS, crosser queue, far movers in their own kernel), with
//   - positions stored as a packed integer cell (10 bits per axis) and FP32
//     offsets in [0, 1), momenta as FP32 (28 bytes per particle instead of 48);
//   - the gather from an FP32 copy of the E/B tile, Boris, advance and the VB
//     split and weights in FP32, in cell-local coordinates;
//   - each FP32 contribution converted (exactly) to FP64 and summed in an FP64
//     (or, in the deterministic mode, exact integer) LDS J tile (ds_add_f64: on gfx950 the FP32 LDS atomic add serializes
//     over the lanes, ~20x the cost of the FP64 one), then added into the
//     FP64 global J.
// This is an extension beyond the paper, which computes in double precision
// throughout (Section 3); the fields, the Yee update and J stay FP64.  Every
// operation is rounded to FP32 as written (fused multiply-adds where written,
// contraction off elsewhere, correctly rounded square roots and divisions),
// so cells, offsets and momenta are reproducible bit for bit by any IEEE FP32
// evaluation of the same expressions.
#include "pic_device.h"
#include "pic_internal.h"

namespace pic {
namespace {

constexpr int kBlock = 512;
constexpr int kCellBits = 10;
constexpr unsigned kCellMask = (1u << kCellBits) - 1u;

__device__ __forceinline__ int near_wrap(int i, int n) {
    i = i < 0 ? i + n : i;
    return i >= n ? i - n : i;
}

__device__ __forceinline__ int tile_node_index(const int org[3], int tx, int ty, int tz, int nx,
                                               int ny, int nz, bool near) {
    if (near)
        return near_wrap(org[0] + tx, nx) +
               nx * (near_wrap(org[1] + ty, ny) + ny * near_wrap(org[2] + tz, nz));
    return wrapi(org[0] + tx, nx) + nx * (wrapi(org[1] + ty, ny) + ny * wrapi(org[2] + tz, nz));
}

__device__ __forceinline__ int xcd_block(int b, int nb) {
    if ((nb & 7) != 0) return b;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

__device__ __forceinline__ unsigned pack_cell(int i, int j, int k) {
    return (unsigned)i | ((unsigned)j << kCellBits) | ((unsigned)k << (2 * kCellBits));
}

__device__ __forceinline__ void unpack_cell(unsigned p, int c[3]) {
    c[0] = (int)(p & kCellMask);
    c[1] = (int)((p >> kCellBits) & kCellMask);
    c[2] = (int)(p >> (2 * kCellBits));
}

struct MArgs {
    Geom g;
    SpeciesM sp;
    PartsM src;             // read: particle i of the new order at perm[i] (or i)
    PartsM dst;             // written: particle i at i
    const unsigned* perm;   // nullptr: identity
    unsigned* keys;         // nullptr: no sort keys wanted
    const int* sc_off;
    const double* EB[6];
    double* J[3];
    unsigned* err;
    unsigned long long* nfar;
    int* far_q;
    unsigned* far_n;
    unsigned* far_n_next;
    DetJ det;               // deterministic mode (hi[0] == nullptr: off)
};

// LDS layouts: FP32 E/B tile of x-pairs: for node (tx, ty, tz) of component
// c with tx < T - 1, the value at 2 tx + EPY ty + EPZ tz + c * ECS and, beside
// it, the difference to the next node in x (what the first lerp of the CIC
// interpolation subtracts, formed once per node instead of once per
// particle; the same FP32 subtraction, so the result is unchanged); FP64 J
// tile, node of component d at d * JC + tx + JPY ty + JPZ tz.  For S = 4,
// h = 1 the pitches are those measured cheapest for the access pattern of a
// round of particles (the E/B plane pitch padded by 4 floats; the J pitches
// 12 / 112 put a half wave of 32 cells on 32 distinct bank pairs).
template <int S, int H>
struct MLayout {
    static constexpr int T = S + 2 * H + 2;
    static constexpr int EPY = 2 * (T - 1);
    static constexpr int EPZ = (S == 4) ? EPY * T + 4 : EPY * T;
    static constexpr int ECS = EPZ * T;
    static constexpr int TJ = S + 2 * H + 3;
    static constexpr int JPY = (S == 4 && H == 1) ? 12 : TJ;
    static constexpr int JPZ = (S == 4 && H == 1) ? 112 : TJ * TJ;
    static constexpr int JC = JPZ * (TJ - 1) + JPY * (TJ - 1) + TJ;
};

__device__ __forceinline__ float lerpf(float a, float b, float f) {
    return __fmaf_rn(f, b - a, a);
}

// Stencil of one axis: stagger 0 -> (c, o); stagger 1/2 -> (c, o - 1/2) if
// o >= 1/2, else (c - 1, o + 1/2).
__device__ __forceinline__ void half_stencil(int c, float o, int& ih, float& fh) {
#pragma clang fp contract(off)
    const bool up = o >= 0.5f;
    ih = up ? c : c - 1;
    fh = up ? o - 0.5f : o + 0.5f;
}

// Eight lattice values of one component (far movers' global gather).
struct Oct8 {
    float v[8];
};

__device__ __forceinline__ float interp8(const Oct8& o, float fx, float fy, float fz) {
#pragma clang fp contract(off)
    const float q00 = lerpf(o.v[0], o.v[1], fx);
    const float q10 = lerpf(o.v[2], o.v[3], fx);
    const float q01 = lerpf(o.v[4], o.v[5], fx);
    const float q11 = lerpf(o.v[6], o.v[7], fx);
    const float r0 = lerpf(q00, q10, fy);
    const float r1 = lerpf(q01, q11, fy);
    return lerpf(r0, r1, fz);
}

// The four x-pairs (value, difference to x + 1) of one component's stencil
// from the LDS tile: one 8-byte read each.
typedef float vf2 __attribute__((ext_vector_type(2)));
struct Pair4 {
    vf2 p[4];
};

template <int PY, int PZ>
__device__ __forceinline__ Pair4 ld_pair4(const float* eb, int base) {
    asm volatile("" : "+v"(base));
    typedef __attribute__((address_space(3))) const volatile vf2 lds_float2;
    const lds_float2* p = (const lds_float2*)(eb + base);
    Pair4 o;
    o.p[0] = p[0];
    o.p[1] = p[PY / 2];
    o.p[2] = p[PZ / 2];
    o.p[3] = p[(PZ + PY) / 2];
    return o;
}

// interp8 on x-pairs: the x lerps take the stored difference.
__device__ __forceinline__ float interp_pairs(const Pair4& o, float fx, float fy, float fz) {
#pragma clang fp contract(off)
    const float q00 = __fmaf_rn(fx, o.p[0].y, o.p[0].x);
    const float q10 = __fmaf_rn(fx, o.p[1].y, o.p[1].x);
    const float q01 = __fmaf_rn(fx, o.p[2].y, o.p[2].x);
    const float q11 = __fmaf_rn(fx, o.p[3].y, o.p[3].x);
    const float r0 = lerpf(q00, q10, fy);
    const float r1 = lerpf(q01, q11, fy);
    return lerpf(r0, r1, fz);
}

// Per-axis stencil: lower index and fraction for stagger 0 (i0, f0) and 1/2.
struct StencilM {
    int i0[3], ih[3];
    float f0[3], fh[3];
};

__device__ __forceinline__ void make_stencil_m(const int c[3], const float o[3], StencilM& st) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        st.i0[d] = c[d];
        st.f0[d] = o[d];
        half_stencil(c[d], o[d], st.ih[d], st.fh[d]);
    }
}

// Gather of the six components from the tile; (off) maps the stencil's cell
// coordinates to tile coordinates.  Yee stagger per component:
// Ex (h,0,0) Ey (0,h,0) Ez (0,0,h) Bx (0,h,h) By (h,0,h) Bz (h,h,0).
template <class L>
__device__ __forceinline__ void gather_tile_m(const float* eb, const StencilM& st,
                                              const int off[3], float E[3], float B[3]) {
    constexpr int PY = L::EPY, PZ = L::EPZ, CS = L::ECS;
    const int x0 = 2 * (st.i0[0] + off[0]), y0 = st.i0[1] + off[1], z0 = st.i0[2] + off[2];
    const int xh = 2 * (st.ih[0] + off[0]), yh = st.ih[1] + off[1], zh = st.ih[2] + off[2];
    Pair4 a = ld_pair4<PY, PZ>(eb, 0 * CS + xh + PY * y0 + PZ * z0);
    Pair4 b = ld_pair4<PY, PZ>(eb, 1 * CS + x0 + PY * yh + PZ * z0);
    E[0] = interp_pairs(a, st.fh[0], st.f0[1], st.f0[2]);
    a = ld_pair4<PY, PZ>(eb, 2 * CS + x0 + PY * y0 + PZ * zh);
    E[1] = interp_pairs(b, st.f0[0], st.fh[1], st.f0[2]);
    b = ld_pair4<PY, PZ>(eb, 3 * CS + x0 + PY * yh + PZ * zh);
    E[2] = interp_pairs(a, st.f0[0], st.f0[1], st.fh[2]);
    a = ld_pair4<PY, PZ>(eb, 4 * CS + xh + PY * y0 + PZ * zh);
    B[0] = interp_pairs(b, st.f0[0], st.fh[1], st.fh[2]);
    b = ld_pair4<PY, PZ>(eb, 5 * CS + xh + PY * yh + PZ * z0);
    B[1] = interp_pairs(a, st.fh[0], st.f0[1], st.fh[2]);
    B[2] = interp_pairs(b, st.fh[0], st.fh[1], st.f0[2]);
}

// Gather of the six components from the global FP64 arrays (far movers);
// the values are rounded to FP32 exactly as the tile copy rounds them.
__device__ __forceinline__ void gather_global_m(const double* const EB[6], const Geom& g,
                                                const StencilM& st, float E[3], float B[3]) {
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    auto F = [&](int comp, int i, int j, int k) {
        return (float)EB[comp][wrapi(i, nx) + nx * (wrapi(j, ny) + ny * wrapi(k, nz))];
    };
    auto comp8 = [&](int comp, int ix, int iy, int iz, float fx, float fy, float fz) {
        Oct8 o;
#pragma unroll
        for (int q = 0; q < 8; ++q) o.v[q] = F(comp, ix + (q & 1), iy + ((q >> 1) & 1), iz + (q >> 2));
        return interp8(o, fx, fy, fz);
    };
    E[0] = comp8(0, st.ih[0], st.i0[1], st.i0[2], st.fh[0], st.f0[1], st.f0[2]);
    E[1] = comp8(1, st.i0[0], st.ih[1], st.i0[2], st.f0[0], st.fh[1], st.f0[2]);
    E[2] = comp8(2, st.i0[0], st.i0[1], st.ih[2], st.f0[0], st.f0[1], st.fh[2]);
    B[0] = comp8(3, st.i0[0], st.ih[1], st.ih[2], st.f0[0], st.fh[1], st.fh[2]);
    B[1] = comp8(4, st.ih[0], st.i0[1], st.ih[2], st.fh[0], st.f0[1], st.fh[2]);
    B[2] = comp8(5, st.ih[0], st.ih[1], st.i0[2], st.fh[0], st.fh[1], st.f0[2]);
}

__device__ __forceinline__ float one_plus_sqf(const float v[3]) {
    return __fmaf_rn(v[2], v[2], __fmaf_rn(v[1], v[1], __fmaf_rn(v[0], v[0], 1.0f)));
}

__device__ __forceinline__ float add_crossf(const float a[3], const float b[3], const float c[3],
                                            int d) {
    const int e = (d + 1) % 3, f = (d + 2) % 3;
    return __fmaf_rn(b[e], c[f], __fmaf_rn(-b[f], c[e], a[d]));
}

// Boris rotation and the cell-local advance o1 = fma((dt/dx_d) u_d, g, o).
// The square roots (of values >= 1) and divisions (by values >= 1, of h, 2
// and 1; |h| is range-checked when a context is created) are correctly
// rounded.
__device__ __forceinline__ void boris_advance_m(const SpeciesM& sp, const float E[3],
                                                const float B[3], float u[3], const float o[3],
                                                float o1[3]) {
#pragma clang fp contract(off)
    const float h = sp.h;
    float um[3], t[3], s[3], up[3], upl[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) um[d] = __fmaf_rn(h, E[d], u[d]);
    const float hg = div_ge1_f32(h, sqrt_ge1_f32(one_plus_sqf(um)));
#pragma unroll
    for (int d = 0; d < 3; ++d) t[d] = hg * B[d];
    const float sf = div_ge1_f32(2.0f, one_plus_sqf(t));
#pragma unroll
    for (int d = 0; d < 3; ++d) s[d] = sf * t[d];
#pragma unroll
    for (int d = 0; d < 3; ++d) up[d] = add_crossf(um, um, t, d);
#pragma unroll
    for (int d = 0; d < 3; ++d) upl[d] = add_crossf(um, up, s, d);
#pragma unroll
    for (int d = 0; d < 3; ++d) u[d] = __fmaf_rn(h, E[d], upl[d]);
    const float gi = div_ge1_f32(1.0f, sqrt_ge1_f32(one_plus_sqf(u)));
#pragma unroll
    for (int d = 0; d < 3; ++d) o1[d] = __fmaf_rn(sp.cdt[d] * u[d], gi, o[d]);
}

// One segment A -> B of a move in cell-local coordinates inside the cell at
// relative corner rc; sink(d, rx, ry, rz, v) adds v to J_d at the edge whose
// integer corner is rc + (offsets), relative to the start cell.
template <class Sink>
__device__ __forceinline__ void vb_segment_m(const float A[3], const float B[3], const int rc[3],
                                             const float jc[3], const Sink& sink) {
#pragma clang fp contract(off)
    float a[3], b[3], dl[3], m[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        a[d] = A[d] - (float)rc[d];
        b[d] = B[d] - (float)rc[d];
        dl[d] = b[d] - a[d];
        m[d] = 0.5f * (a[d] + b[d]);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
        const int p = e1 < e2 ? e1 : e2;
        const int r = e1 < e2 ? e2 : e1;
        const float cross = (dl[p] * dl[r]) * (1.0f / 12.0f);
        const float flux = jc[d] * dl[d];
#pragma unroll
        for (int bp = 0; bp < 2; ++bp) {
            const float wp = bp ? m[p] : 1.0f - m[p];
#pragma unroll
            for (int br = 0; br < 2; ++br) {
                const float wr = br ? m[r] : 1.0f - m[r];
                const float W = wp * wr + ((bp == br) ? cross : -cross);
                int o[3] = {0, 0, 0};
                o[p] = bp;
                o[r] = br;
                sink(d, rc[0] + o[0], rc[1] + o[1], rc[2] + o[2], flux * W);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

__device__ __forceinline__ void cswapf(float& ta, int& da, float& tb, int& db) {
    const bool sw = (tb < ta) || (tb == ta && db < da);
    const float t = sw ? tb : ta;
    const int d = sw ? db : da;
    tb = sw ? ta : tb;
    db = sw ? da : db;
    ta = t;
    da = d;
}

// VB split of a cell-local move o0 -> o1 (o0 in [0,1)^3, o1 in (-1,2)^3) at the
// cell planes it crosses, in order of crossing time (ties x, y, z); junction
// points are o0 + t (o1 - o0) with the crossing coordinate set to the plane.
template <class Sink>
__device__ __forceinline__ void vb_move_m(const float o0[3], const float o1[3], const float jc[3],
                                          const Sink& sink) {
#pragma clang fp contract(off)
    float dv[3], pl[3], t[3];
    int c1[3], dm[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        dv[d] = o1[d] - o0[d];
        c1[d] = (int)floorf(o1[d]);
        pl[d] = (float)(c1[d] > 0 ? c1[d] : 0);
        t[d] = (c1[d] != 0) ? (pl[d] - o0[d]) / dv[d] : __builtin_huge_valf();
        dm[d] = d;
    }
    int left = (c1[0] != 0) + (c1[1] != 0) + (c1[2] != 0);
    cswapf(t[0], dm[0], t[1], dm[1]);
    cswapf(t[1], dm[1], t[2], dm[2]);
    cswapf(t[0], dm[0], t[1], dm[1]);
    float A[3] = {o0[0], o0[1], o0[2]};
    int rc[3] = {0, 0, 0};
#pragma unroll 1
    for (;;) {
        float B[3];
#pragma unroll
        for (int d = 0; d < 3; ++d)
            B[d] = (left == 0) ? o1[d] : ((dm[0] == d) ? pl[d] : __fmaf_rn(t[0], dv[d], o0[d]));
        vb_segment_m(A, B, rc, jc, sink);
        if (left == 0) break;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            A[d] = B[d];
            if (dm[0] == d) rc[d] = c1[d];
        }
        t[0] = t[1];
        dm[0] = dm[1];
        t[1] = t[2];
        dm[1] = dm[2];
        --left;
    }
}

// The twelve J contributions of a move that stays in its cell, ordered
// (d, bp, br); add(j, v) receives them.
template <class Add>
__device__ __forceinline__ void vb_single_m(const float o0[3], const float o1[3],
                                            const float jc[3], const Add& add) {
#pragma clang fp contract(off)
    float dl[3], m[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        dl[d] = o1[d] - o0[d];
        m[d] = 0.5f * (o0[d] + o1[d]);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
        const int p = e1 < e2 ? e1 : e2;
        const int r = e1 < e2 ? e2 : e1;
        const float cross = (dl[p] * dl[r]) * (1.0f / 12.0f);
        const float flux = jc[d] * dl[d];
        const float wp0 = 1.0f - m[p], wr0 = 1.0f - m[r];
        add(4 * d + 0, flux * (wp0 * wr0 + cross));
        add(4 * d + 1, flux * (wp0 * m[r] - cross));
        add(4 * d + 2, flux * (m[p] * wr0 - cross));
        add(4 * d + 3, flux * (m[p] * m[r] + cross));
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <int PY, int PZ, int JC>
__device__ __forceinline__ constexpr int jt_off_m(int j) {
    const int d = j >> 2, bp = (j >> 1) & 1, br = j & 1;
    const int sp = (d == 0) ? PY : 1;
    const int sr = (d == 2) ? PY : PZ;
    return d * JC + bp * sp + br * sr;
}

// New cell and offset after the move: s = floor(o1), c = (c + s) mod n,
// o = o1 - s; an offset that rounds to 1 becomes 0 in the next cell.
__device__ __forceinline__ void cell_update(const int c[3], const float o1[3], const int n[3],
                                            int cn[3], float on[3]) {
#pragma clang fp contract(off)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float s = floorf(o1[d]);
        int v = c[d] + (int)s;
        v = v < 0 ? v + n[d] : (v >= n[d] ? v - n[d] : v);
        float w = o1[d] - s;
        if (w >= 1.0f) {
            w = 0.0f;
            v = (v + 1 == n[d]) ? 0 : v + 1;
        }
        cn[d] = v;
        on[d] = w;
    }
}

template <int S>
__device__ __forceinline__ unsigned sort_key_m(const Geom& g, const int c[3]) {
    const int sc = c[0] / S + g.ns[0] * (c[1] / S + g.ns[1] * (c[2] / S));
    const int loc = c[0] % S + S * (c[1] % S + S * (c[2] % S));
    return (unsigned)(sc * S * S * S + loc);
}

__device__ __forceinline__ unsigned sort_key_m_rt(const Geom& g, const int c[3]) {
    const int S = g.S;
    const int sc = c[0] / S + g.ns[0] * (c[1] / S + g.ns[1] * (c[2] / S));
    const int loc = c[0] % S + S * (c[1] % S + S * (c[2] % S));
    return (unsigned)(sc * S * S * S + loc);
}

__device__ __forceinline__ bool finite3f(float a, float b, float c) {
    return isfinite(a) && isfinite(b) && isfinite(c);
}

template <int S, int H, bool GATHER, bool DET>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6)))
push_mixed_kernel(const MArgs a) {
    using L = MLayout<S, H>;
    constexpr int T = L::T, T2 = T * T, T3 = T2 * T;
    constexpr int TJ = L::TJ;
    constexpr int JPY = L::JPY, JPZ = L::JPZ, JC = L::JC;
    constexpr int kWaves = kBlock / 64;
    constexpr int QCAP = 28;
    __shared__ __attribute__((aligned(16))) float eb[6 * L::ECS];
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
    __shared__ float qb[kWaves][6][QCAP];
    __shared__ int qk[kWaves][QCAP];

    const int sc = xcd_block(blockIdx.x, gridDim.x);
    const int p0 = a.sc_off[sc], p1 = a.sc_off[sc + 1];
    if (p0 >= p1) return;
    if (DET && p1 - p0 > kDetMaxPerSupercell) {
        if (threadIdx.x == 0) atomicOr(a.err, ERR_DETCAP);
        return;
    }

    const Geom& g = a.g;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const int nn[3] = {nx, ny, nz};
    const int sx = sc % g.ns[0];
    const int syz = sc / g.ns[0];
    const int sy = syz % g.ns[1], sz = syz / g.ns[1];
    const int base[3] = {sx * S, sy * S, sz * S};
    const int org[3] = {base[0] - H - 1, base[1] - H - 1, base[2] - H - 1};
    const bool near = nx >= H + 2 && ny >= H + 2 && nz >= H + 2;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const unsigned long long lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    // the first particle's loads go out before the tile loads: the two
    // latencies overlap
    unsigned ncell = 0u;
    float nxt[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    auto ld7 = [&](int ip, unsigned& cp, float o[6]) {
        const unsigned j = GATHER ? a.perm[ip] : (unsigned)ip;
        const unsigned b = j * 4u;
        cp = *(const unsigned*)((const char*)a.src.cell + b);
        o[0] = *(const float*)((const char*)a.src.ox + b);
        o[1] = *(const float*)((const char*)a.src.oy + b);
        o[2] = *(const float*)((const char*)a.src.oz + b);
        o[3] = *(const float*)((const char*)a.src.ux + b);
        o[4] = *(const float*)((const char*)a.src.uy + b);
        o[5] = *(const float*)((const char*)a.src.uz + b);
    };
    {
        const int ip = p0 + (int)threadIdx.x;
        if (ip < p1) ld7(ip, ncell, nxt);
    }

    // tile of x-pairs: the values first (the last node of a row in the
    // difference slot of the pair before it), then the differences
    for (int r = threadIdx.x; r < T3; r += kBlock) {
        const int tz = r / T2, ty = (r / T) % T, tx = r % T;
        const int gi = tile_node_index(org, tx, ty, tz, nx, ny, nz, near);
        const int li = (tx < T - 1 ? 2 * tx : 2 * T - 3) + L::EPY * ty + L::EPZ * tz;
#pragma unroll
        for (int c = 0; c < 6; ++c) eb[c * L::ECS + li] = (float)a.EB[c][gi];
    }
    for (int t = threadIdx.x; t < JT_BYTES / 4; t += kBlock) ((int*)jraw)[t] = 0;
    __syncthreads();
    for (int r = threadIdx.x; r < T3; r += kBlock) {
        const int tz = r / T2, ty = (r / T) % T, tx = r % T;
        if (tx < T - 1) {
            const int li = 2 * tx + L::EPY * ty + L::EPZ * tz;
            const int ln = tx < T - 2 ? li + 2 : li + 1;
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const float v0 = eb[c * L::ECS + li], v1 = eb[c * L::ECS + ln];
                eb[c * L::ECS + li + 1] = v1 - v0;
            }
        }
    }
    __syncthreads();

    // relative cell of c inside the tile window [-H, S+H), periodic
    auto relcell = [&](const int c[3], int rel[3]) {
        bool in = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int r = c[d] - base[d];
            if (r >= S + H)
                r -= nn[d];
            else if (r < -H)
                r += nn[d];
            rel[d] = r;
            in = in && (r >= -H) && (r < S + H);
        }
        return in;
    };
    // general move of a particle whose start cell sits at tile key `key`
    auto deposit_tile = [&](int key, const float o0[3], const float o1[3]) {
        vb_move_m(o0, o1, a.sp.jc, [&](int d, int rx, int ry, int rz, float v) {
            jadd(d * JC + key + rx + JPY * ry + JPZ * rz, (double)v);
        });
    };
    auto drain = [&](int cnt) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < cnt) {
            const float q0[3] = {qb[wv][0][lane], qb[wv][1][lane], qb[wv][2][lane]};
            const float q1[3] = {qb[wv][3][lane], qb[wv][4][lane], qb[wv][5][lane]};
            deposit_tile(qk[wv][lane], q0, q1);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };

    int qcount = 0;
    for (int pb = p0; pb < p1; pb += kBlock) {
        const int ip = pb + (int)threadIdx.x;
        const bool valid = ip < p1;
        const unsigned cp = ncell;
        float o0[3] = {nxt[0], nxt[1], nxt[2]};
        float u[3] = {nxt[3], nxt[4], nxt[5]};
        {
            const int in = ip + kBlock;
            if (in < p1) ld7(in, ncell, nxt);
        }
        bool crosser = false, far = false;
        float o1[3] = {0.f, 0.f, 0.f};
        int key = 0;
        // every lane stores (see push_deposit_kernel): lanes without a pushed
        // particle store to the spare slot
        unsigned o = a.dst.spare;
        int cn[3] = {0, 0, 0};
        float on[3] = {0.f, 0.f, 0.f};
        if (valid) {
            int c[3], rel[3];
            unpack_cell(cp, c);
            const bool inside = relcell(c, rel);
            far = !inside;
            bool ok = true;
            if (inside) {
                StencilM st;
                make_stencil_m(c, o0, st);
                int off[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) off[d] = rel[d] + H + 1 - c[d];
                float E[3], B[3];
                gather_tile_m<L>(eb, st, off, E, B);
                boris_advance_m(a.sp, E, B, u, o0, o1);
                ok = finite3f(u[0], u[1], u[2]) && finite3f(o1[0], o1[1], o1[2]);
            }
            if (!ok) {
                atomicOr(a.err, ERR_NONFINITE);
            } else if (inside) {
                key = (rel[0] + H + 1) + JPY * (rel[1] + H + 1) + JPZ * (rel[2] + H + 1);
                const bool single = floorf(o1[0]) == 0.0f && floorf(o1[1]) == 0.0f &&
                                    floorf(o1[2]) == 0.0f;
                if (single) {
                    vb_single_m(o0, o1, a.sp.jc, [&](int j, float v) {
                        jadd(key + jt_off_m<JPY, JPZ, JC>(j), (double)v);
                    });
                } else {
                    crosser = true;
                }
                cell_update(c, o1, nn, cn, on);
                o = (unsigned)ip;
            }
        }
        {
            const unsigned b = o * 4u;
            *(unsigned*)((char*)a.dst.cell + b) = pack_cell(cn[0], cn[1], cn[2]);
            *(float*)((char*)a.dst.ox + b) = on[0];
            *(float*)((char*)a.dst.oy + b) = on[1];
            *(float*)((char*)a.dst.oz + b) = on[2];
            *(float*)((char*)a.dst.ux + b) = u[0];
            *(float*)((char*)a.dst.uy + b) = u[1];
            *(float*)((char*)a.dst.uz + b) = u[2];
            if (a.keys && o != a.dst.spare) a.keys[o] = sort_key_m<S>(g, cn);
        }
        {
            const unsigned long long fm = __ballot(far);
            if (fm) {
                const int lead = __ffsll((long long)fm) - 1;
                unsigned fb = 0;
                if (lane == lead) fb = atomicAdd(a.far_n, (unsigned)__popcll(fm));
                fb = (unsigned)__builtin_amdgcn_readlane((int)fb, lead);
                if (far) a.far_q[fb + (unsigned)__popcll(fm & lt_mask)] = ip;
            }
        }
        {
            const unsigned long long cm = __ballot(crosser);
            const int nnew = __popcll(cm);
            if (nnew > QCAP) {
                if (crosser) deposit_tile(key, o0, o1);
            } else if (nnew > 0) {
                if (qcount + nnew > QCAP) {
                    drain(qcount);
                    qcount = 0;
                }
                if (crosser) {
                    const int slot = qcount + __popcll(cm & lt_mask);
                    qb[wv][0][slot] = o0[0];
                    qb[wv][1][slot] = o0[1];
                    qb[wv][2][slot] = o0[2];
                    qb[wv][3][slot] = o1[0];
                    qb[wv][4][slot] = o1[1];
                    qb[wv][5][slot] = o1[2];
                    qk[wv][slot] = key;
                }
                qcount += nnew;
            }
        }
    }
    if (qcount > 0) drain(qcount);
    __syncthreads();

    constexpr int TJ2 = TJ * TJ, TJ3 = TJ2 * TJ;
    for (int r = threadIdx.x; r < TJ3; r += kBlock) {
        const int tz = r / TJ2, ty = (r / TJ) % TJ, tx = r % TJ;
        const int li = tx + JPY * ty + JPZ * tz;
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

// Particles beyond their supercell's tile window: global gather (FP64 values
// rounded to FP32), the same FP32 push, global FP64 atomics.
__global__ void __launch_bounds__(kBlock) far_mixed_kernel(const MArgs a) {
    const unsigned n = *a.far_n;
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.far_n_next = 0u;
    const Geom& g = a.g;
    const int nn[3] = {g.n[0], g.n[1], g.n[2]};
    unsigned long long cnt = 0;
    // queue entry i goes to workgroup i mod gridDim: a short queue (the usual
    // case) spreads one particle per workgroup over the CUs instead of
    // filling the waves of the first workgroup
    for (unsigned i = threadIdx.x * gridDim.x + blockIdx.x; i < n; i += gridDim.x * kBlock) {
        const int ip = a.far_q[i];
        const unsigned j = a.perm ? a.perm[ip] : (unsigned)ip;
        int c[3];
        unpack_cell(a.src.cell[j], c);
        const float o0[3] = {a.src.ox[j], a.src.oy[j], a.src.oz[j]};
        float u[3] = {a.src.ux[j], a.src.uy[j], a.src.uz[j]};
        StencilM st;
        make_stencil_m(c, o0, st);
        float E[3], B[3], o1[3];
        gather_global_m(a.EB, g, st, E, B);
        boris_advance_m(a.sp, E, B, u, o0, o1);
        if (!(finite3f(u[0], u[1], u[2]) && finite3f(o1[0], o1[1], o1[2]))) {
            atomicOr(a.err, ERR_NONFINITE);
            continue;
        }
        vb_move_m(o0, o1, a.sp.jc, [&](int d, int rx, int ry, int rz, float v) {
            const int gi = wrapi(c[0] + rx, nn[0]) +
                           nn[0] * (wrapi(c[1] + ry, nn[1]) + nn[1] * wrapi(c[2] + rz, nn[2]));
            if (a.det.hi[0]) {
                unsigned long long h;
                int l;
                det_split((double)v, a.det.scale, h, l);
                atomicAdd(&a.det.hi[d][gi], h);
                atomicAdd((unsigned long long*)&a.det.lo[d][gi], (unsigned long long)(long long)l);
            } else {
                unsafeAtomicAdd(&a.J[d][gi], (double)v);
            }
        });
        int cn[3];
        float on[3];
        cell_update(c, o1, nn, cn, on);
        a.dst.cell[ip] = pack_cell(cn[0], cn[1], cn[2]);
        a.dst.ox[ip] = on[0];
        a.dst.oy[ip] = on[1];
        a.dst.oz[ip] = on[2];
        a.dst.ux[ip] = u[0];
        a.dst.uy[ip] = u[1];
        a.dst.uz[ip] = u[2];
        if (a.keys) a.keys[ip] = sort_key_m_rt(g, cn);
        cnt += 1;
    }
    if (cnt) atomicAdd(a.nfar, cnt);
}

// Conversion of FP64 positions and momenta into the packed form, with the
// validity check of a load (ERR_BADPOS) and the sort key of every particle.
__global__ void __launch_bounds__(256) to_mixed_kernel(Geom g, int n, const double* x,
                                                       const double* y, const double* z,
                                                       const double* ux, const double* uy,
                                                       const double* uz, PartsM dst,
                                                       unsigned* key, unsigned* err) {
#pragma clang fp contract(off)
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const double p[3] = {x[i], y[i], z[i]};
        const double uu[3] = {ux[i], uy[i], uz[i]};
        bool ok = true;
        int c[3];
        float o[3], uf[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            uf[d] = (float)uu[d];
            const bool in = p[d] >= 0.0 && p[d] < (double)g.n[d];
            ok = ok && in && isfinite(uf[d]);
            const double fl = in ? floor(p[d]) : 0.0;
            int ci = (int)fl;
            float of = in ? (float)(p[d] - fl) : 0.0f;
            if (of >= 1.0f) {
                of = 0.0f;
                ci = (ci + 1 == g.n[d]) ? 0 : ci + 1;
            }
            c[d] = ci;
            o[d] = of;
        }
        if (!ok) atomicOr(err, ERR_BADPOS);
        dst.cell[i] = pack_cell(c[0], c[1], c[2]);
        dst.ox[i] = o[0];
        dst.oy[i] = o[1];
        dst.oz[i] = o[2];
        dst.ux[i] = uf[0];
        dst.uy[i] = uf[1];
        dst.uz[i] = uf[2];
        key[i] = sort_key_m_rt(g, c);
    }
}

__global__ void __launch_bounds__(256) to_double_kernel(int n, PartsM src, double* x, double* y,
                                                        double* z, double* ux, double* uy,
                                                        double* uz) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        int c[3];
        unpack_cell(src.cell[i], c);
        x[i] = (double)c[0] + (double)src.ox[i];
        y[i] = (double)c[1] + (double)src.oy[i];
        z[i] = (double)c[2] + (double)src.oz[i];
        ux[i] = (double)src.ux[i];
        uy[i] = (double)src.uy[i];
        uz[i] = (double)src.uz[i];
    }
}

__global__ void __launch_bounds__(256) permute_mixed_kernel(int n, const unsigned* perm,
                                                            PartsM src, PartsM dst) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const unsigned j = perm[i];
        dst.cell[i] = src.cell[j];
        dst.ox[i] = src.ox[j];
        dst.oy[i] = src.oy[j];
        dst.oz[i] = src.oz[j];
        dst.ux[i] = src.ux[j];
        dst.uy[i] = src.uy[j];
        dst.uz[i] = src.uz[j];
        dst.id[i] = src.id[j];
    }
}

int grid256(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    return b < 1 ? 1 : (int)b;
}

template <int S, int H>
hipError_t launch_m(const MArgs& args, hipStream_t s) {
    const bool det = args.det.hi[0] != nullptr;
    const dim3 grid(args.g.nsc), block(kBlock);
    if (args.perm && det)
        hipLaunchKernelGGL((push_mixed_kernel<S, H, true, true>), grid, block, 0, s, args);
    else if (args.perm)
        hipLaunchKernelGGL((push_mixed_kernel<S, H, true, false>), grid, block, 0, s, args);
    else if (det)
        hipLaunchKernelGGL((push_mixed_kernel<S, H, false, true>), grid, block, 0, s, args);
    else
        hipLaunchKernelGGL((push_mixed_kernel<S, H, false, false>), grid, block, 0, s, args);
    return hipGetLastError();
}

template <int S, int H>
constexpr int lds_bytes_m(bool det) {
    return 6 * MLayout<S, H>::ECS * (int)sizeof(float) + 3 * MLayout<S, H>::JC * (det ? 12 : 8) +
           (kBlock / 64) * 7 * 28 * 4;
}

MArgs make_margs(const Geom& g, const SpeciesM& sp, const PartsM& src, const PartsM& dst,
                 const unsigned* perm, unsigned* keys, const int* sc_off, const Fields& f,
                 double* const J[3], unsigned* err, unsigned long long* nfar, int* far_q,
                 unsigned* far_n, unsigned* far_n_next, const DetJ& det) {
    MArgs a;
    a.det = det;
    a.g = g;
    a.sp = sp;
    a.src = src;
    a.dst = dst;
    a.perm = perm;
    a.keys = keys;
    a.sc_off = sc_off;
    for (int c = 0; c < 3; ++c) {
        a.EB[c] = f.E[c];
        a.EB[3 + c] = f.B[c];
        a.J[c] = J[c];
    }
    a.err = err;
    a.nfar = nfar;
    a.far_q = far_q;
    a.far_n = far_n;
    a.far_n_next = far_n_next;
    return a;
}

}  // namespace

#define PIC_SH_TABLE_M(X) \
    X(1, 1) X(1, 2) X(2, 1) X(2, 2) X(3, 1) X(4, 1) X(4, 2) X(5, 1) X(6, 1)

int push_mixed_lds_bytes(const Geom& g, bool det) {
#define PIC_X(s_, h_) if (g.S == s_ && g.h == h_) return lds_bytes_m<s_, h_>(det);
    PIC_SH_TABLE_M(PIC_X)
#undef PIC_X
    return -1;
}

hipError_t launch_push_mixed(const Geom& g, const SpeciesM& sp, const PartsM& src,
                             const PartsM& dst, const unsigned* perm, unsigned* keys,
                             const int* sc_off, const Fields& f, double* const J[3],
                             unsigned* err, unsigned long long* nfar, int* far_q,
                             unsigned* far_n, unsigned* far_n_next, const DetJ& det,
                             hipStream_t s) {
    const MArgs args = make_margs(g, sp, src, dst, perm, keys, sc_off, f, J, err, nfar, far_q,
                                  far_n, far_n_next, det);
    if (g.nsc <= 0) return hipSuccess;
#define PIC_X(s_, h_) if (g.S == s_ && g.h == h_) return launch_m<s_, h_>(args, s);
    PIC_SH_TABLE_M(PIC_X)
#undef PIC_X
    return hipErrorInvalidValue;
}

hipError_t launch_far_mixed(const Geom& g, const SpeciesM& sp, const PartsM& src,
                            const PartsM& dst, const unsigned* perm, unsigned* keys,
                            const Fields& f, double* const J[3], unsigned* err,
                            unsigned long long* nfar, int* far_q, unsigned* far_n,
                            unsigned* far_n_next, const DetJ& det, hipStream_t s) {
    const MArgs args = make_margs(g, sp, src, dst, perm, keys, nullptr, f, J, err, nfar, far_q,
                                  far_n, far_n_next, det);
    hipLaunchKernelGGL(far_mixed_kernel, dim3(256), dim3(kBlock), 0, s, args);
    return hipGetLastError();
}

hipError_t launch_to_mixed(const Geom& g, int64_t n, const double* const x[6], const PartsM& dst,
                           unsigned* keys, unsigned* err, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(to_mixed_kernel, dim3(grid256(n)), dim3(256), 0, s, g, (int)n, x[0], x[1],
                       x[2], x[3], x[4], x[5], dst, keys, err);
    return hipGetLastError();
}

hipError_t launch_to_double(int64_t n, const PartsM& src, double* const x[6], hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(to_double_kernel, dim3(grid256(n)), dim3(256), 0, s, (int)n, src, x[0],
                       x[1], x[2], x[3], x[4], x[5]);
    return hipGetLastError();
}

hipError_t launch_permute_mixed(int64_t n, const unsigned* perm, const PartsM& src,
                                const PartsM& dst, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(permute_mixed_kernel, dim3(grid256(n)), dim3(256), 0, s, (int)n, perm, src,
                       dst);
    return hipGetLastError();
}

}  // namespace pic
