// Adjoint (reverse-mode derivative) of the PIC step, FP64.
//
// The forward step is: gather E/B at each particle (cloud-in-cell on the Yee
// lattice), Boris push, straight advance, Villasenor-Buneman deposit of the
// move, periodic wrap, then the Yee update with that current (stage order of
// Section 2; schemes of Section 3).  Its adjoint, per step in reverse:
//
//   fields  (linear):  lE -= (dt/2) C_B lB;  lB += dt C_E lE;  lJ = -dt lE;
//                      lE -= (dt/2) C_B lB
//     (C_E forward-difference curl E -> B lattice, C_B backward-difference
//     curl B -> E lattice; on the periodic lattice C_B^T = C_E);
//   particles:         the vector-Jacobian product of gather -> Boris ->
//                      advance -> deposit, one particle per thread, with the
//                      deposit's gradient read from lJ and the transposed
//                      interpolation summed per workgroup in an LDS tile
//                      (its particles are consecutive in the supercell-sorted
//                      order, so their stencils share a small box) and added
//                      into lE / lB with one FP64 atomic per node;
//   re-sort:           the adjoint of a particle moves back to the particle's
//                      slot before the re-sort.
//
// The kernels read the forward state of the step (positions, momenta and the
// fields at its start), which the host recomputes from checkpoints.  Apart
// from the transposed interpolation they use global memory directly: the
// adjoint runs once per gradient, not in the stepping loop.
#include "pic_device.h"
#include "pic_internal.h"

namespace pic {
namespace {

constexpr int kAdjBlock = 256;
// Edge (nodes) of the LDS tile of the transposed interpolation.
constexpr int kAdjTile = 10;

int grid_for(int64_t n) {
    int64_t b = (n + kAdjBlock - 1) / kAdjBlock;
    if (b > 65536) b = 65536;
    return (int)(b < 1 ? 1 : b);
}

__device__ __forceinline__ int lin3(const Geom& g, int i, int j, int k) {
    return wrapi(i, g.n[0]) + g.n[0] * (wrapi(j, g.n[1]) + g.n[1] * wrapi(k, g.n[2]));
}

// lE -= coef * C_B lB at every E point; when lJ is given, first lJ = jcoef * lE.
__global__ void adj_e_kernel(Geom g, double* lEx, double* lEy, double* lEz, const double* lBx,
                             const double* lBy, const double* lBz, double coef, double* lJx,
                             double* lJy, double* lJz, double jcoef) {
#pragma clang fp contract(off)
    const double dx = g.dx[0], dy = g.dx[1], dz = g.dx[2];
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < g.ncell; c += gridDim.x * blockDim.x) {
        const int i = c % g.n[0];
        const int j = (c / g.n[0]) % g.n[1];
        const int k = c / (g.n[0] * g.n[1]);
        const double cx = (lBz[c] - lBz[lin3(g, i, j - 1, k)]) / dy -
                          (lBy[c] - lBy[lin3(g, i, j, k - 1)]) / dz;
        const double cy = (lBx[c] - lBx[lin3(g, i, j, k - 1)]) / dz -
                          (lBz[c] - lBz[lin3(g, i - 1, j, k)]) / dx;
        const double cz = (lBy[c] - lBy[lin3(g, i - 1, j, k)]) / dx -
                          (lBx[c] - lBx[lin3(g, i, j - 1, k)]) / dy;
        const double ex = lEx[c], ey = lEy[c], ez = lEz[c];
        if (lJx) {
            lJx[c] = jcoef * ex;
            lJy[c] = jcoef * ey;
            lJz[c] = jcoef * ez;
        }
        lEx[c] = ex - coef * cx;
        lEy[c] = ey - coef * cy;
        lEz[c] = ez - coef * cz;
    }
}

// lB += coef * C_E lE at every B point.
__global__ void adj_b_kernel(Geom g, const double* lEx, const double* lEy, const double* lEz,
                             double* lBx, double* lBy, double* lBz, double coef) {
#pragma clang fp contract(off)
    const double dx = g.dx[0], dy = g.dx[1], dz = g.dx[2];
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < g.ncell; c += gridDim.x * blockDim.x) {
        const int i = c % g.n[0];
        const int j = (c / g.n[0]) % g.n[1];
        const int k = c / (g.n[0] * g.n[1]);
        const double cx = (lEz[lin3(g, i, j + 1, k)] - lEz[c]) / dy -
                          (lEy[lin3(g, i, j, k + 1)] - lEy[c]) / dz;
        const double cy = (lEx[lin3(g, i, j, k + 1)] - lEx[c]) / dz -
                          (lEz[lin3(g, i + 1, j, k)] - lEz[c]) / dx;
        const double cz = (lEy[lin3(g, i + 1, j, k)] - lEy[c]) / dx -
                          (lEx[lin3(g, i, j + 1, k)] - lEx[c]) / dy;
        lBx[c] = lBx[c] + coef * cx;
        lBy[c] = lBy[c] + coef * cy;
        lBz[c] = lBz[c] + coef * cz;
    }
}

struct AdjArgs {
    Geom g;
    SpeciesC sp;
    int n;
    const double* x[3];     // state at the start of the step
    const double* u[3];
    const double* EB[6];    // fields at the start of the step
    const double* lJ[3];
    double* lx[3];          // adjoint of the state: end of step in, start of step out
    double* lu[3];
    double* lEB[6];         // accumulated (atomics)
};

// Yee stagger of component c along dimension d is 1/2 for
// Ex: x; Ey: y; Ez: z; Bx: y, z; By: x, z; Bz: x, y.
__device__ __forceinline__ bool half_stag(int c, int d) {
    return c < 3 ? (c == d) : (c - 3 != d);
}

struct Cic {
    int i[3];
    double f[3];
    double v[8];   // v[a + 2 b + 4 e] = F[i + (a, b, e)]
};

// Stencil position of component c at x: lower node and fractions.
__device__ __forceinline__ void cic_place(int c, const double x[3], Cic& p) {
#pragma clang fp contract(off)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double xi = half_stag(c, d) ? x[d] - 0.5 : x[d];
        const double fl = floor(xi);
        p.i[d] = (int)fl;
        p.f[d] = xi - fl;
    }
}

__device__ __forceinline__ void cic_load(const Geom& g, const double* F, int c, const double x[3],
                                         Cic& p) {
    cic_place(c, x, p);
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a)
                p.v[a + 2 * b + 4 * e] = F[lin3(g, p.i[0] + a, p.i[1] + b, p.i[2] + e)];
}

__device__ __forceinline__ double wgt(int a, double f) { return a ? f : 1.0 - f; }
__device__ __forceinline__ double dwgt(int a) { return a ? 1.0 : -1.0; }

// value (nested fused lerps, as the forward gather) and gradient in x
__device__ __forceinline__ double cic_value_grad(const Cic& p, double gr[3]) {
#pragma clang fp contract(off)
    gr[0] = gr[1] = gr[2] = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const double v = p.v[a + 2 * b + 4 * e];
                gr[0] += dwgt(a) * wgt(b, p.f[1]) * wgt(e, p.f[2]) * v;
                gr[1] += wgt(a, p.f[0]) * dwgt(b) * wgt(e, p.f[2]) * v;
                gr[2] += wgt(a, p.f[0]) * wgt(b, p.f[1]) * dwgt(e) * v;
            }
    return cic8([&](int a, int b, int e) { return p.v[a + 2 * b + 4 * e]; }, p.f[0], p.f[1],
                p.f[2]);
}

__device__ __forceinline__ void cic_scatter(const Geom& g, double* F, const Cic& p, double lF) {
#pragma clang fp contract(off)
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a)
                atomicAdd(F + lin3(g, p.i[0] + a, p.i[1] + b, p.i[2] + e),
                          lF * wgt(a, p.f[0]) * wgt(b, p.f[1]) * wgt(e, p.f[2]));
}

// The same into an LDS tile of edge kAdjTile whose node (0, 0, 0) is the
// unwrapped lattice node lo (every node of the stencil lies in the tile).
__device__ __forceinline__ void cic_scatter_tile(double* T, const int lo[3], const Cic& p,
                                                 double lF) {
#pragma clang fp contract(off)
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a)
                atomicAdd(T + (p.i[0] + a - lo[0]) +
                              kAdjTile * ((p.i[1] + b - lo[1]) + kAdjTile * (p.i[2] + e - lo[2])),
                          lF * wgt(a, p.f[0]) * wgt(b, p.f[1]) * wgt(e, p.f[2]));
}

// Gradient of <lJ, VB(A -> B in cell)> with respect to A and B: with a, b
// the local end points, dl = b - a and m = (a + b)/2, direction d with
// transverse axes p < r contributes
//   jc_d dl_d sum L[bp][br] (w_bp(m_p) w_br(m_r) +- dl_p dl_r / 12).
__device__ __forceinline__ void vb_segment_grad(const Geom& g, const double* const lJ[3],
                                                const int cell[3], const double A[3],
                                                const double B[3], const double jc[3],
                                                double gA[3], double gB[3]) {
#pragma clang fp contract(off)
    double a[3], b[3], dl[3], m[3], gdl[3] = {0.0, 0.0, 0.0}, gm[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        a[d] = A[d] - (double)cell[d];
        b[d] = B[d] - (double)cell[d];
        dl[d] = b[d] - a[d];
        m[d] = 0.5 * (a[d] + b[d]);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
        const int p = e1 < e2 ? e1 : e2;
        const int r = e1 < e2 ? e2 : e1;
        double L[2][2];
#pragma unroll
        for (int bp = 0; bp < 2; ++bp)
#pragma unroll
            for (int br = 0; br < 2; ++br) {
                int idx[3] = {cell[0], cell[1], cell[2]};
                idx[p] += bp;
                idx[r] += br;
                L[bp][br] = lJ[d][lin3(g, idx[0], idx[1], idx[2])];
            }
        double P = 0.0, dmp = 0.0, dmr = 0.0, K = 0.0;
#pragma unroll
        for (int bp = 0; bp < 2; ++bp)
#pragma unroll
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
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        gA[d] = -gdl[d] + 0.5 * gm[d];
        gB[d] = gdl[d] + 0.5 * gm[d];
    }
}

// Gradient of <lJ, VB(x0 -> x1)> with respect to x0 and x1 (accumulated).
// The move is split exactly as the forward deposit splits it: crossing
// times t_d = (plane_d - x0_d) / (x1_d - x0_d), ordered by time then
// dimension; the junction k is x0 + t_k (x1 - x0) with its crossing
// coordinate on the plane, and its Jacobian chains the junction gradient back
// to x0 and x1.
__device__ __forceinline__ void vb_move_grad(const Geom& g, const double* const lJ[3],
                                             const double x0[3], const double x1[3],
                                             const double jc[3], double gx0[3], double gx1[3]) {
#pragma clang fp contract(off)
    double dv[3], pl[3], t[3];
    int dm[3], c0[3], c1[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        c0[d] = (int)floor(x0[d]);
        c1[d] = (int)floor(x1[d]);
        dv[d] = x1[d] - x0[d];
        const int p = c0[d] > c1[d] ? c0[d] : c1[d];
        pl[d] = (double)p;
        t[d] = (c1[d] != c0[d]) ? (pl[d] - x0[d]) / dv[d] : __builtin_huge_val();
        dm[d] = d;
    }
    const int left = (c1[0] != c0[0]) + (c1[1] != c0[1]) + (c1[2] != c0[2]);
    cswap(t[0], dm[0], t[1], dm[1]);
    cswap(t[1], dm[1], t[2], dm[2]);
    cswap(t[0], dm[0], t[1], dm[1]);
    double A[3] = {x0[0], x0[1], x0[2]};
    int cell[3] = {c0[0], c0[1], c0[2]};
    double gPrev[3] = {0.0, 0.0, 0.0};   // gradient at the current segment's start point
    // one segment at a time: its twelve lJ loads are the only ones in flight
#pragma unroll 1
    for (int k = 0; k < 4; ++k) {
        if (k > left) break;
        const int kk = k < 3 ? k : 2;      // crossing k exists only for k < left <= 3
        double B[3];
#pragma unroll
        for (int d = 0; d < 3; ++d)
            B[d] = (k == left) ? x1[d] : ((dm[kk] == d) ? pl[d] : x0[d] + t[kk] * dv[d]);
        double gA[3], gB[3];
        vb_segment_grad(g, lJ, cell, A, B, jc, gA, gB);
        // start point of this segment: x0 (k == 0) or junction k - 1
#pragma unroll
        for (int d = 0; d < 3; ++d) gPrev[d] += gA[d];
        if (k == 0) {
#pragma unroll
            for (int d = 0; d < 3; ++d) gx0[d] += gPrev[d];
        } else {
            const int e = dm[k - 1];
            const double tk = t[k - 1];
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                if (f == e) continue;
                const double G = gPrev[f];
                gx0[f] += G * (1.0 - tk);
                gx1[f] += G * tk;
                gx0[e] += G * dv[f] * (tk - 1.0) / dv[e];
                gx1[e] += G * dv[f] * (-tk) / dv[e];
            }
        }
        // end point: junction k (its gradient completes with the next
        // segment's start) or x1
#pragma unroll
        for (int d = 0; d < 3; ++d) gPrev[d] = gB[d];
        if (k == left) {
#pragma unroll
            for (int d = 0; d < 3; ++d) gx1[d] += gPrev[d];
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            A[d] = B[d];
            if (k < left && dm[kk] == d) cell[d] = c1[d];
        }
    }
}

__device__ __forceinline__ double dot3(const double a[3], const double b[3]) {
#pragma clang fp contract(off)
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double o[3]) {
#pragma clang fp contract(off)
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

__global__ void __launch_bounds__(kAdjBlock) particle_adjoint_kernel(AdjArgs A) {
#pragma clang fp contract(off)
    const Geom& g = A.g;
    // The particles of a workgroup are consecutive in the stored order, which
    // is sorted by supercell: their interpolation nodes usually lie in a small
    // box.  Then the transposed interpolation is summed in an LDS tile over
    // that box and added into lE / lB once per node; otherwise (a box wider
    // than the tile, e.g. across the periodic boundary) each particle adds
    // into global memory directly.
    constexpr int TB = kAdjTile, TB3 = TB * TB * TB;
    __shared__ double ltile[6][TB3];
    __shared__ int box[6];
    for (int p0 = blockIdx.x * kAdjBlock; p0 < A.n; p0 += gridDim.x * kAdjBlock) {
        const int p = p0 + (int)threadIdx.x;
        const bool valid = p < A.n;
        if (threadIdx.x < 3) box[threadIdx.x] = 0x7fffffff;
        else if (threadIdx.x < 6) box[threadIdx.x] = -0x7fffffff;
        __syncthreads();
        double x0[3] = {0.0, 0.0, 0.0}, u0[3] = {0.0, 0.0, 0.0};
        if (valid) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                x0[d] = A.x[d][p];
                u0[d] = A.u[d][p];
            }
            // nodes of every stagger: floor(x) - 1 .. floor(x) + 1
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int c = (int)floor(x0[d]);
                atomicMin(&box[d], c - 1);
                atomicMax(&box[3 + d], c + 1);
            }
        }
        __syncthreads();
        const int lo[3] = {box[0], box[1], box[2]};
        const bool tiled = box[3] - lo[0] < TB && box[4] - lo[1] < TB && box[5] - lo[2] < TB;
        if (tiled)
            for (int t = threadIdx.x; t < 6 * TB3; t += kAdjBlock) (&ltile[0][0])[t] = 0.0;
        __syncthreads();
        if (valid) {
        // forward values (the stencils are recomputed for the scatter below,
        // so that only the values and their gradients stay live)
        double F[6], dF[6][3];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            Cic cp;
            cic_load(g, A.EB[c], c, x0, cp);
            F[c] = cic_value_grad(cp, dF[c]);
        }
        const double* E = F;
        const double* Bf = F + 3;
        const double h = A.sp.hq;
        double um[3], t[3], s[3], up[3], upl[3], u1[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) um[d] = __fma_rn(h, E[d], u0[d]);
        const double gm = sqrt_ge1(one_plus_sq(um));
        const double hg = div_ge1(h, gm);
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
        for (int d = 0; d < 3; ++d) u1[d] = __fma_rn(h, E[d], upl[d]);
        const double gi = div_ge1(1.0, sqrt_ge1(one_plus_sq(u1)));
        double x1[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) x1[d] = __fma_rn(g.cdt[d] * u1[d], gi, x0[d]);

        // reverse: deposit and advance
        double lxs[3] = {A.lx[0][p], A.lx[1][p], A.lx[2][p]};   // wrap: derivative 1
        double lu1[3] = {A.lu[0][p], A.lu[1][p], A.lu[2][p]};
        double gx0[3] = {0.0, 0.0, 0.0}, gx1[3] = {0.0, 0.0, 0.0};
        vb_move_grad(g, A.lJ, x0, x1, A.sp.jc, gx0, gx1);
#pragma unroll
        for (int d = 0; d < 3; ++d) lxs[d] += gx1[d];
        double lx0[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) lx0[d] = lxs[d] + gx0[d];
        double v[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) v[d] = g.cdt[d] * lxs[d];
        const double uv = dot3(u1, v);
#pragma unroll
        for (int d = 0; d < 3; ++d) lu1[d] += gi * v[d] - u1[d] * uv * gi * gi * gi;
        // reverse: Boris
        double lE[3], lB[3], lum[3], lup[3], ls[3], lt[3], tmp[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            lE[d] = h * lu1[d];
            lum[d] = lu1[d];
        }
        cross3(s, lu1, lup);
        cross3(lu1, up, ls);
#pragma unroll
        for (int d = 0; d < 3; ++d) lum[d] += lup[d];
        cross3(t, lup, tmp);
#pragma unroll
        for (int d = 0; d < 3; ++d) lum[d] += tmp[d];
        cross3(lup, um, lt);
        const double lst = dot3(ls, t);
#pragma unroll
        for (int d = 0; d < 3; ++d) lt[d] += sf * ls[d] - sf * sf * lst * t[d];
#pragma unroll
        for (int d = 0; d < 3; ++d) lB[d] = hg * lt[d];
        const double lhg = dot3(lt, Bf);
        const double lgm = -(hg / gm) * lhg;
#pragma unroll
        for (int d = 0; d < 3; ++d) lum[d] += (lgm / gm) * um[d];
#pragma unroll
        for (int d = 0; d < 3; ++d) lE[d] += h * lum[d];
        // reverse: interpolation
        const double lF[6] = {lE[0], lE[1], lE[2], lB[0], lB[1], lB[2]};
#pragma unroll
        for (int c = 0; c < 6; ++c) {
#pragma unroll
            for (int d = 0; d < 3; ++d) lx0[d] += lF[c] * dF[c][d];
            Cic cp;
            cic_place(c, x0, cp);
            if (tiled)
                cic_scatter_tile(ltile[c], lo, cp, lF[c]);
            else
                cic_scatter(g, A.lEB[c], cp, lF[c]);
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            A.lx[d][p] = lx0[d];
            A.lu[d][p] = lum[d];
        }
        }  // valid
        __syncthreads();
        if (tiled) {
            for (int t = threadIdx.x; t < TB3; t += kAdjBlock) {
                const int tx = t % TB, ty = (t / TB) % TB, tz = t / (TB * TB);
                const int gi = lin3(g, lo[0] + tx, lo[1] + ty, lo[2] + tz);
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    const double v = ltile[c][t];
                    if (v != 0.0) atomicAdd(A.lEB[c] + gi, v);
                }
            }
        }
        __syncthreads();   // the tile and the box are reused by the next range
    }
}

// dst[perm[i]] = src[i] for six arrays: the adjoint of the re-sort gather
// dst_new[i] = src_old[perm[i]].
struct Six {
    double* a[6];
};

__global__ void unpermute_kernel(int n, const unsigned* perm, Six src, Six dst) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const unsigned o = perm[i];
#pragma unroll
        for (int k = 0; k < 6; ++k) dst.a[k][o] = src.a[k][i];
    }
}

}  // namespace

hipError_t launch_fdtd_adjoint(const Geom& g, double* const lE[3], double* const lB[3],
                               double* const lJ[3], hipStream_t s) {
    const int nb = grid_for(g.ncell);
    const double h = 0.5 * g.dt;
    hipLaunchKernelGGL(adj_e_kernel, dim3(nb), dim3(kAdjBlock), 0, s, g, lE[0], lE[1], lE[2],
                       lB[0], lB[1], lB[2], h, (double*)nullptr, (double*)nullptr,
                       (double*)nullptr, 0.0);
    hipLaunchKernelGGL(adj_b_kernel, dim3(nb), dim3(kAdjBlock), 0, s, g, lE[0], lE[1], lE[2],
                       lB[0], lB[1], lB[2], g.dt);
    hipLaunchKernelGGL(adj_e_kernel, dim3(nb), dim3(kAdjBlock), 0, s, g, lE[0], lE[1], lE[2],
                       lB[0], lB[1], lB[2], h, lJ[0], lJ[1], lJ[2], -g.dt);
    return hipGetLastError();
}

hipError_t launch_particle_adjoint(const Geom& g, const SpeciesC& sp, int64_t n,
                                   const double* const state[6], const double* const EB[6],
                                   const double* const lJ[3], double* const lam[6],
                                   double* const lEB[6], hipStream_t s) {
    if (n <= 0) return hipSuccess;
    AdjArgs a;
    a.g = g;
    a.sp = sp;
    a.n = (int)n;
    for (int d = 0; d < 3; ++d) {
        a.x[d] = state[d];
        a.u[d] = state[3 + d];
        a.lJ[d] = lJ[d];
        a.lx[d] = lam[d];
        a.lu[d] = lam[3 + d];
    }
    for (int c = 0; c < 6; ++c) {
        a.EB[c] = EB[c];
        a.lEB[c] = lEB[c];
    }
    hipLaunchKernelGGL(particle_adjoint_kernel, dim3(grid_for(n)), dim3(kAdjBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_unpermute(int64_t n, const unsigned* perm, double* const src[6],
                            double* const dst[6], hipStream_t s) {
    if (n <= 0) return hipSuccess;
    Six a, b;
    for (int k = 0; k < 6; ++k) {
        a.a[k] = src[k];
        b.a[k] = dst[k];
    }
    hipLaunchKernelGGL(unpermute_kernel, dim3(grid_for(n)), dim3(kAdjBlock), 0, s, (int)n, perm,
                       a, b);
    return hipGetLastError();
}

}  // namespace pic
