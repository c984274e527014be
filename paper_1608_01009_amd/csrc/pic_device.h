// Device helpers shared by the forward particle kernels and the adjoint:
// periodic index wrap, cloud-in-cell interpolation, the crossing-order
// compare-exchange of the Villasenor-Buneman split, correctly rounded square
// root and division for the operand ranges of the Boris push, the Boris
// rotation with the position advance, the periodic position wrap and the
// interpolation stencil.
#pragma once

#include "pic_internal.h"

namespace pic {
namespace {

__device__ __forceinline__ int wrapi(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

// Cloud-in-cell (trilinear) interpolation of one component as nested linear
// interpolation, x first, then y, then z, with lerp(a, b, f) = fma(f, b - a, a);
// ld(a, b, c) returns the lattice value at offset (a, b, c).
template <class Load>
__device__ __forceinline__ double cic8(const Load& ld, double fx, double fy, double fz) {
#pragma clang fp contract(off)
    double r[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        double q[2];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const double f0 = ld(0, b, c), f1 = ld(1, b, c);
            q[b] = __fma_rn(fx, f1 - f0, f0);
        }
        r[c] = __fma_rn(fy, q[1] - q[0], q[0]);
    }
    return __fma_rn(fz, r[1] - r[0], r[0]);
}

// Compare-exchange of (time, dimension) pairs ordered by time, then dimension.
__device__ __forceinline__ void cswap(double& ta, int& da, double& tb, int& db) {
    const bool sw = (tb < ta) || (tb == ta && db < da);
    const double t = sw ? tb : ta;
    const int d = sw ? db : da;
    tb = sw ? ta : tb;
    db = sw ? da : db;
    ta = t;
    da = d;
}

// Square root of x >= 1 (finite), correctly rounded: the reciprocal square
// root estimate refined by Newton steps and two fused residual corrections.
// These are the operations of the general IEEE FP64 square root of gfx9 less
// its range scaling, which is the identity for x >= 1, so the result is the
// same bit for bit.
__device__ __forceinline__ double sqrt_ge1(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = __fma_rn(-h, g, 0.5);
    g = __fma_rn(g, r, g);
    h = __fma_rn(h, r, h);
    double d = __fma_rn(-g, g, x);
    g = __fma_rn(d, h, g);
    d = __fma_rn(-g, g, x);
    return __fma_rn(d, h, g);
}

// a / b, correctly rounded, for 1 <= b < 2^1000 and a = 0 or
// 2^-900 < |a| < 2^900: reciprocal estimate, two Newton steps, quotient and
// one fused residual correction.  Again the operations of the general IEEE
// FP64 division less its range scaling and special-case fix-up, neither of
// which acts on operands in these ranges.
__device__ __forceinline__ double div_ge1(double a, double b) {
    double r = __builtin_amdgcn_rcp(b);
    double e = __fma_rn(-b, r, 1.0);
    r = __fma_rn(r, e, r);
    e = __fma_rn(-b, r, 1.0);
    r = __fma_rn(r, e, r);
    const double q = a * r;
    e = __fma_rn(-b, q, a);
    return __fma_rn(e, r, q);
}

// FP32 square root of x >= 1 (finite), correctly rounded: the hardware
// square root (within one unit in the last place) moved to the neighbour
// above or below when the fused residual against it has the right sign.
// These are the operations of the general IEEE FP32 square root of gfx9 less
// its scaling of tiny operands and its special-value select, neither of which
// acts for x >= 1, so the result is the same bit for bit.
__device__ __forceinline__ float sqrt_ge1_f32(float x) {
    const float s = __builtin_amdgcn_sqrtf(x);
    const float dn = __int_as_float(__float_as_int(s) - 1);
    const float up = __int_as_float(__float_as_int(s) + 1);
    float r = __fmaf_rn(-dn, s, x) <= 0.0f ? dn : s;
    r = __fmaf_rn(-up, s, x) > 0.0f ? up : r;
    return r;
}

// FP32 a / b, correctly rounded, for 1 <= b < 2^64 and a = 0 or
// 2^-60 < |a| < 2^60: reciprocal estimate, one Newton step, quotient and two
// fused residual corrections; the operations of the general IEEE FP32
// division of gfx9 less its operand scaling and special-case fix-up, which do
// not act for quotients in the normal range.
__device__ __forceinline__ float div_ge1_f32(float a, float b) {
    float r = __builtin_amdgcn_rcpf(b);
    r = __fmaf_rn(__fmaf_rn(-b, r, 1.0f), r, r);
    float q = a * r;
    q = __fmaf_rn(__fmaf_rn(-b, q, a), r, q);
    return __fmaf_rn(__fmaf_rn(-b, q, a), r, q);
}

__device__ __forceinline__ double one_plus_sq(const double v[3]) {
    return __fma_rn(v[2], v[2], __fma_rn(v[1], v[1], __fma_rn(v[0], v[0], 1.0)));
}

// component d of a + b x c, as two fused multiply-adds
__device__ __forceinline__ double add_cross(const double a[3], const double b[3],
                                            const double c[3], int d) {
    const int e = (d + 1) % 3, f = (d + 2) % 3;
    return __fma_rn(b[e], c[f], __fma_rn(-b[f], c[e], a[d]));
}

// Boris rotation (half E kick, B rotation, half E kick) and the straight
// position advance x1 = x0 + (dt/dx_d) u_d / gamma.  Every sum of products is
// a chain of fused multiply-adds in a fixed order; gamma- >= 1 and
// 1 + |t|^2 >= 1 keep the square roots and divisions in the ranges of
// sqrt_ge1 and div_ge1 (|q dt / 2m| is range-checked when a context is
// created).
__device__ __forceinline__ void boris_advance(const SpeciesC& sp, const Geom& g, const double E[3],
                                              const double Bf[3], double u[3], const double x0[3],
                                              double x1[3]) {
#pragma clang fp contract(off)
    const double h = sp.hq;
    double um[3], t[3], s[3], up[3], upl[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) um[d] = __fma_rn(h, E[d], u[d]);
    const double hg = div_ge1(h, sqrt_ge1(one_plus_sq(um)));
#pragma unroll
    for (int d = 0; d < 3; ++d) t[d] = hg * Bf[d];
    const double sf = div_ge1(2.0, one_plus_sq(t));
#pragma unroll
    for (int d = 0; d < 3; ++d) s[d] = sf * t[d];
#pragma unroll
    for (int d = 0; d < 3; ++d) up[d] = add_cross(um, um, t, d);
#pragma unroll
    for (int d = 0; d < 3; ++d) upl[d] = add_cross(um, up, s, d);
#pragma unroll
    for (int d = 0; d < 3; ++d) u[d] = __fma_rn(h, E[d], upl[d]);
    const double gi = div_ge1(1.0, sqrt_ge1(one_plus_sq(u)));
#pragma unroll
    for (int d = 0; d < 3; ++d) x1[d] = __fma_rn(g.cdt[d] * u[d], gi, x0[d]);
}

__device__ __forceinline__ double wrap_coord(double v, double L) {
#pragma clang fp contract(off)
    if (v >= L)
        v = v - L;
    else if (v < 0.0)
        v = v + L;
    if (v == L) v = 0.0;
    return v;
}

// Interpolation stencil of one position: for stagger 0 and 1/2 per axis the
// lower lattice index and the fractional offset.
struct Stencil {
    int i0[3], ih[3];
    double f0[3], fh[3];
};

__device__ __forceinline__ void make_stencil(const double x[3], const double fl[3], Stencil& st) {
#pragma clang fp contract(off)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        st.i0[d] = (int)fl[d];
        st.f0[d] = x[d] - fl[d];
        const double xh = x[d] - 0.5;
        const double flh = floor(xh);
        st.ih[d] = (int)flh;
        st.fh[d] = xh - flh;
    }
}

}  // namespace
}  // namespace pic
