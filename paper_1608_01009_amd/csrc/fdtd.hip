// Maxwell integration on the Yee lattice (stage 1 of the PIC step of
// arXiv:1608.01009, Section 2), with B kept at integer time levels:
//   B' = B - dt/2 curl E;  E' = E + dt (curl B' - J);  B'' = B' - dt/2 curl E'.
// One fused kernel: each workgroup owns a block of 8^3 cells and stages E
// (block plus a halo of one below and two above), B (one below and one
// above) and J in LDS, computes B' on the block plus halo, E' on the block
// plus one layer above, then B'' on the block, and writes E' and B'' to a
// second pair of arrays (the update is out of place, so neighbouring blocks
// read only the old values).  It also clears the J buffer that the next step
// deposits into.  The differences are written in the order of the textbook
// stencils with contraction off, so E and B are reproducible bit for bit
// given the same J.
#include "pic_internal.h"

namespace pic {
namespace {

constexpr int kBlock = 256;

struct FArgs {
    int n[3];
    int nb[3];          // blocks per dimension
    double dt, hdt;
    double dx[3];
    const double* E[3];
    const double* B[3];
    const double* J[3];
    double* Eo[3];
    double* Bo[3];
    double* Jc[3];
};

constexpr int YB = 8;                 // block edge in cells
constexpr int YT = 256;               // threads per workgroup
constexpr int NE = YB + 3;            // E tile edge: cells lo-1 .. hi+1
constexpr int NBt = YB + 2;           // B tile edge: cells lo-1 .. hi
constexpr int NE1 = YB + 1;           // E' tile edge: cells lo .. hi

// i mod n; the tile coordinates lie in [-n, 2n) when n >= 3 (`near`)
__device__ __forceinline__ int pwrap(int i, int n, bool near) {
    if (near) {
        i = i < 0 ? i + n : i;
        return i >= n ? i - n : i;
    }
    int r = i % n;
    return r < 0 ? r + n : r;
}

// UNIT: every dx_d == 1, where the divisions by dx_d are the identity and
// are left out (the results are the same bit for bit).
template <bool UNIT>
__device__ __forceinline__ double ddx(double v, double dx) {
#pragma clang fp contract(off)
    return UNIT ? v : v / dx;
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Give each XCD a contiguous range of blocks (with x fastest, whole
// layers of blocks along z), so that the halos of neighbouring blocks in x and
// y are fetched from HBM once per XCD rather than once per block.
__device__ __forceinline__ int yee_xcd_block(int b, int nb) {
    if ((nb & 7) != 0) return b;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

template <bool UNIT>
__global__ void __launch_bounds__(YT) yee_kernel(const FArgs a) {
#pragma clang fp contract(off)
    __shared__ double e0[3][NE * NE * NE];
    __shared__ double bt[3][NBt * NBt * NBt];
    __shared__ double e1[3][NE1 * NE1 * NE1];
    const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
    const int b = yee_xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int bxi = b % a.nb[0], byz = b / a.nb[0];
    const int byi = byz % a.nb[1], bzi = byz / a.nb[1];
    const int lo[3] = {bxi * YB, byi * YB, bzi * YB};
    const double dx0 = a.dx[0], dx1 = a.dx[1], dx2 = a.dx[2];
    // block coordinates reach at most 2 cells beyond [0, n) on either side
    const bool near = nx >= YB + 2 && ny >= YB + 2 && nz >= YB + 2;
    auto gidx = [&](int x, int y, int z) {
        return pwrap(x, nx, near) + nx * (pwrap(y, ny, near) + ny * pwrap(z, nz, near));
    };
    // J at the E' points of this thread, fetched before the staging barrier
    constexpr int NJ = (NE1 * NE1 * NE1 + YT - 1) / YT;
    double jv[NJ][3];
#pragma unroll
    for (int k = 0; k < NJ; ++k) {
        const int t = threadIdx.x + k * YT;
        if (t < NE1 * NE1 * NE1) {
            const int tx = t % NE1, ty = (t / NE1) % NE1, tz = t / (NE1 * NE1);
            const int g = gidx(lo[0] + tx, lo[1] + ty, lo[2] + tz);
            jv[k][0] = a.J[0][g];
            jv[k][1] = a.J[1][g];
            jv[k][2] = a.J[2][g];
        }
    }
    // stage E (origin lo-1, edge NE) and B (origin lo-1, edge NBt): all
    // global loads are issued before the first LDS store
    constexpr int KE = (NE * NE * NE + YT - 1) / YT;
    constexpr int KB = (NBt * NBt * NBt + YT - 1) / YT;
    double ev[KE][3], bv[KB][3];
#pragma unroll
    for (int k = 0; k < KE; ++k) {
        const int t = threadIdx.x + k * YT;
        if (t < NE * NE * NE) {
            const int tx = t % NE, ty = (t / NE) % NE, tz = t / (NE * NE);
            const int g = gidx(lo[0] - 1 + tx, lo[1] - 1 + ty, lo[2] - 1 + tz);
#pragma unroll
            for (int c = 0; c < 3; ++c) ev[k][c] = a.E[c][g];
        }
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        const int t = threadIdx.x + k * YT;
        if (t < NBt * NBt * NBt) {
            const int tx = t % NBt, ty = (t / NBt) % NBt, tz = t / (NBt * NBt);
            const int g = gidx(lo[0] - 1 + tx, lo[1] - 1 + ty, lo[2] - 1 + tz);
#pragma unroll
            for (int c = 0; c < 3; ++c) bv[k][c] = a.B[c][g];
        }
    }
#pragma unroll
    for (int k = 0; k < KE; ++k) {
        const int t = threadIdx.x + k * YT;
        if (t < NE * NE * NE) {
#pragma unroll
            for (int c = 0; c < 3; ++c) e0[c][t] = ev[k][c];
        }
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        const int t = threadIdx.x + k * YT;
        if (t < NBt * NBt * NBt) {
#pragma unroll
            for (int c = 0; c < 3; ++c) bt[c][t] = bv[k][c];
        }
    }
    __syncthreads();
    // B' = B - dt/2 curl E on cells lo-1 .. hi (E tile index = B tile index
    // with the same origin, E tile edge NE)
    for (int t = threadIdx.x; t < NBt * NBt * NBt; t += YT) {
        const int tx = t % NBt, ty = (t / NBt) % NBt, tz = t / (NBt * NBt);
        const int e = tx + NE * (ty + NE * tz);
        const double ex = e0[0][e], ey = e0[1][e], ez = e0[2][e];
        const int ip = e + 1, jp = e + NE, kp = e + NE * NE;
        const double cx = ddx<UNIT>(e0[2][jp] - ez, dx1) - ddx<UNIT>(e0[1][kp] - ey, dx2);
        const double cy = ddx<UNIT>(e0[0][kp] - ex, dx2) - ddx<UNIT>(e0[2][ip] - ez, dx0);
        const double cz = ddx<UNIT>(e0[1][ip] - ey, dx0) - ddx<UNIT>(e0[0][jp] - ex, dx1);
        bt[0][t] = bt[0][t] - a.hdt * cx;
        bt[1][t] = bt[1][t] - a.hdt * cy;
        bt[2][t] = bt[2][t] - a.hdt * cz;
    }
    __syncthreads();
    // E' = E + dt (curl B' - J) on cells lo .. hi
#pragma unroll
    for (int k = 0; k < NJ; ++k) {
        const int t = threadIdx.x + k * YT;
        if (t >= NE1 * NE1 * NE1) break;
        const int tx = t % NE1, ty = (t / NE1) % NE1, tz = t / (NE1 * NE1);
        const int bb = (tx + 1) + NBt * ((ty + 1) + NBt * (tz + 1));
        const int e = (tx + 1) + NE * ((ty + 1) + NE * (tz + 1));
        const double bx = bt[0][bb], by = bt[1][bb], bz = bt[2][bb];
        const int im = bb - 1, jm = bb - NBt, km = bb - NBt * NBt;
        const double cx = ddx<UNIT>(bz - bt[2][jm], dx1) - ddx<UNIT>(by - bt[1][km], dx2);
        const double cy = ddx<UNIT>(bx - bt[0][km], dx2) - ddx<UNIT>(bz - bt[2][im], dx0);
        const double cz = ddx<UNIT>(by - bt[1][im], dx0) - ddx<UNIT>(bx - bt[0][jm], dx1);
        e1[0][t] = e0[0][e] + a.dt * (cx - jv[k][0]);
        e1[1][t] = e0[1][e] + a.dt * (cy - jv[k][1]);
        e1[2][t] = e0[2][e] + a.dt * (cz - jv[k][2]);
    }
    __syncthreads();
    // B'' = B' - dt/2 curl E' on the block; write E', B'', clear J.  The
    // stores are non-temporal: nothing in this launch reads them again, and
    // less dirty data in L2 shortens the write-back at the end of the launch.
    for (int t = threadIdx.x; t < YB * YB * YB; t += YT) {
        const int tx = t % YB, ty = (t / YB) % YB, tz = t / (YB * YB);
        const int cx_ = lo[0] + tx, cy_ = lo[1] + ty, cz_ = lo[2] + tz;
        if (cx_ >= nx || cy_ >= ny || cz_ >= nz) continue;
        const int g = cx_ + nx * (cy_ + ny * cz_);
        const int e = tx + NE1 * (ty + NE1 * tz);
        const int bb = (tx + 1) + NBt * ((ty + 1) + NBt * (tz + 1));
        const double ex = e1[0][e], ey = e1[1][e], ez = e1[2][e];
        const int ip = e + 1, jp = e + NE1, kp = e + NE1 * NE1;
        const double cx = ddx<UNIT>(e1[2][jp] - ez, dx1) - ddx<UNIT>(e1[1][kp] - ey, dx2);
        const double cy = ddx<UNIT>(e1[0][kp] - ex, dx2) - ddx<UNIT>(e1[2][ip] - ez, dx0);
        const double cz = ddx<UNIT>(e1[1][ip] - ey, dx0) - ddx<UNIT>(e1[0][jp] - ex, dx1);
        __builtin_nontemporal_store(bt[0][bb] - a.hdt * cx, &a.Bo[0][g]);
        __builtin_nontemporal_store(bt[1][bb] - a.hdt * cy, &a.Bo[1][g]);
        __builtin_nontemporal_store(bt[2][bb] - a.hdt * cz, &a.Bo[2][g]);
        __builtin_nontemporal_store(ex, &a.Eo[0][g]);
        __builtin_nontemporal_store(ey, &a.Eo[1][g]);
        __builtin_nontemporal_store(ez, &a.Eo[2][g]);
        __builtin_nontemporal_store(0.0, &a.Jc[0][g]);
        __builtin_nontemporal_store(0.0, &a.Jc[1][g]);
        __builtin_nontemporal_store(0.0, &a.Jc[2][g]);
    }
}

__global__ void __launch_bounds__(kBlock) zero_kernel(double* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        p[i] = 0.0;
}

int grid_for(int64_t n) {
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b > 65536) b = 65536;
    return b < 1 ? 1 : (int)b;
}

}  // namespace

namespace {

// ---- absorbing x boundaries --------------------------------------------
// Plain global-memory passes (see include/pic.h for the boundary scheme):
// half B out of place, E with the Mur planes and the laser sheet, half B in
// place.  x indices stay inside [0, n0); y and z wrap.

struct AbsArgs {
    int n[3];
    double dt, hdt;
    double dx[3];
    int plane;          // laser sheet node plane, -1: none
    double laser;       // Jy added on that plane this step
};

__device__ __forceinline__ int lin_abs(const AbsArgs& a, int i, int j, int k) {
    j = j < 0 ? j + a.n[1] : (j >= a.n[1] ? j - a.n[1] : j);
    k = k < 0 ? k + a.n[2] : (k >= a.n[2] ? k - a.n[2] : k);
    return i + a.n[0] * (j + a.n[1] * k);
}

// Bo = B - dt/2 curl E; the slot n0-1 of By, Bz (outside) is zero.  Bo may
// equal B (each thread reads and writes its own cell only).  Jy, when not
// null, receives the laser sheet's current on its plane: the E update has
// already consumed it (as a term of its own), and the stored J of the step
// includes the source.  No kernel of the update reads J after the E pass, so
// that write cannot race with a read.
__global__ void __launch_bounds__(kBlock) abs_half_b_kernel(AbsArgs a, const double* Ex,
                                                           const double* Ey, const double* Ez,
                                                           const double* Bx, const double* By,
                                                           const double* Bz, double* Box,
                                                           double* Boy, double* Boz, double* Jy) {
#pragma clang fp contract(off)
    const int nx = a.n[0], ncell = a.n[0] * a.n[1] * a.n[2];
    const double dx = a.dx[0], dy = a.dx[1], dz = a.dx[2];
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncell; c += gridDim.x * blockDim.x) {
        const int i = c % nx, j = (c / nx) % a.n[1], k = c / (nx * a.n[1]);
        if (Jy && i == a.plane) Jy[c] = Jy[c] + a.laser;
        const double cx = (Ez[lin_abs(a, i, j + 1, k)] - Ez[c]) / dy -
                          (Ey[lin_abs(a, i, j, k + 1)] - Ey[c]) / dz;
        Box[c] = Bx[c] - a.hdt * cx;
        if (i == nx - 1) {
            Boy[c] = 0.0;
            Boz[c] = 0.0;
            continue;
        }
        const double cy = (Ex[lin_abs(a, i, j, k + 1)] - Ex[c]) / dz -
                          (Ez[lin_abs(a, i + 1, j, k)] - Ez[c]) / dx;
        const double cz = (Ey[lin_abs(a, i + 1, j, k)] - Ey[c]) / dx -
                          (Ex[lin_abs(a, i, j + 1, k)] - Ex[c]) / dy;
        Boy[c] = By[c] - a.hdt * cy;
        Boz[c] = Bz[c] - a.hdt * cz;
    }
}

struct Ey2 {
    double y, z;
};

// E_y, E_z after the curl update at an inside plane 1 <= i <= n0-2 (the laser
// sheet's current added to the deposited Jy on its plane; J itself is only
// read here)
__device__ __forceinline__ Ey2 e_inside(const AbsArgs& a, int i, int j, int k,
                                        const double* const E[3], const double* const B[3],
                                        const double* const J[3]) {
#pragma clang fp contract(off)
    const int c = lin_abs(a, i, j, k);
    const double dx = a.dx[0], dy = a.dx[1], dz = a.dx[2];
    const double cy = (B[0][c] - B[0][lin_abs(a, i, j, k - 1)]) / dz -
                      (B[2][c] - B[2][lin_abs(a, i - 1, j, k)]) / dx;
    const double cz = (B[1][c] - B[1][lin_abs(a, i - 1, j, k)]) / dx -
                      (B[0][c] - B[0][lin_abs(a, i, j - 1, k)]) / dy;
    double jy = J[1][c];
    if (i == a.plane) jy = jy + a.laser;
    return {E[1][c] + a.dt * (cy - jy), E[2][c] + a.dt * (cz - J[2][c])};
}

__global__ void __launch_bounds__(kBlock) abs_e_kernel(AbsArgs a, const double* E0,
                                                      const double* E1, const double* E2,
                                                      const double* B0, const double* B1,
                                                      const double* B2, const double* J0,
                                                      const double* J1, const double* J2,
                                                      double* Eo0, double* Eo1,
                                                      double* Eo2, double* Jc0, double* Jc1,
                                                      double* Jc2) {
#pragma clang fp contract(off)
    const int nx = a.n[0], ncell = a.n[0] * a.n[1] * a.n[2];
    const double dy = a.dx[1], dz = a.dx[2];
    const double kmur = (a.dt - a.dx[0]) / (a.dt + a.dx[0]);
    const double* const E[3] = {E0, E1, E2};
    const double* const B[3] = {B0, B1, B2};
    const double* const J[3] = {J0, J1, J2};
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncell; c += gridDim.x * blockDim.x) {
        const int i = c % nx, j = (c / nx) % a.n[1], k = c / (nx * a.n[1]);
        if (i < nx - 1) {
            const double cx = (B[2][c] - B[2][lin_abs(a, i, j - 1, k)]) / dy -
                              (B[1][c] - B[1][lin_abs(a, i, j, k - 1)]) / dz;
            Eo0[c] = E[0][c] + a.dt * (cx - J[0][c]);
        } else {
            Eo0[c] = 0.0;
        }
        if (i == 0 || i == nx - 1) {
            // first-order Mur: the inside neighbour's new value, recomputed here
            const int in = (i == 0) ? 1 : nx - 2;
            const int cn = lin_abs(a, in, j, k);
            const Ey2 en = e_inside(a, in, j, k, E, B, J);
            Eo1[c] = E[1][cn] + kmur * (en.y - E[1][c]);
            Eo2[c] = E[2][cn] + kmur * (en.z - E[2][c]);
        } else {
            const Ey2 e = e_inside(a, i, j, k, E, B, J);
            Eo1[c] = e.y;
            Eo2[c] = e.z;
        }
        Jc0[c] = 0.0;
        Jc1[c] = 0.0;
        Jc2[c] = 0.0;
    }
}

}  // namespace

hipError_t launch_fdtd_absorbing(const Geom& g, const Fields& f, const Fields& fo,
                                 double* const J[3], double* const Jclear[3], int laser_plane,
                                 double laser_j, hipStream_t s) {
    AbsArgs a;
    for (int d = 0; d < 3; ++d) {
        a.n[d] = g.n[d];
        a.dx[d] = g.dx[d];
    }
    a.dt = g.dt;
    a.hdt = 0.5 * g.dt;
    a.plane = laser_plane;
    a.laser = laser_j;
    int nb = (g.ncell + kBlock - 1) / kBlock;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(abs_half_b_kernel, dim3(nb), dim3(kBlock), 0, s, a, f.E[0], f.E[1],
                       f.E[2], f.B[0], f.B[1], f.B[2], fo.B[0], fo.B[1], fo.B[2],
                       (double*)nullptr);
    hipLaunchKernelGGL(abs_e_kernel, dim3(nb), dim3(kBlock), 0, s, a, f.E[0], f.E[1], f.E[2],
                       fo.B[0], fo.B[1], fo.B[2], J[0], J[1], J[2], fo.E[0], fo.E[1], fo.E[2],
                       Jclear[0], Jclear[1], Jclear[2]);
    hipLaunchKernelGGL(abs_half_b_kernel, dim3(nb), dim3(kBlock), 0, s, a, fo.E[0], fo.E[1],
                       fo.E[2], fo.B[0], fo.B[1], fo.B[2], fo.B[0], fo.B[1], fo.B[2],
                       laser_plane >= 0 ? J[1] : (double*)nullptr);
    return hipGetLastError();
}

hipError_t launch_fdtd(const Geom& g, const Fields& f, const Fields& fo, double* const J[3],
                       double* const Jclear[3], hipStream_t s) {
    FArgs a;
    for (int d = 0; d < 3; ++d) {
        a.n[d] = g.n[d];
        a.nb[d] = (g.n[d] + YB - 1) / YB;
        a.dx[d] = g.dx[d];
        a.E[d] = f.E[d];
        a.B[d] = f.B[d];
        a.Eo[d] = fo.E[d];
        a.Bo[d] = fo.B[d];
        a.J[d] = J[d];
        a.Jc[d] = Jclear[d];
    }
    a.dt = g.dt;
    a.hdt = 0.5 * g.dt;
    const int nb = a.nb[0] * a.nb[1] * a.nb[2];
    if (g.dx[0] == 1.0 && g.dx[1] == 1.0 && g.dx[2] == 1.0)
        hipLaunchKernelGGL(yee_kernel<true>, dim3(nb), dim3(YT), 0, s, a);
    else
        hipLaunchKernelGGL(yee_kernel<false>, dim3(nb), dim3(YT), 0, s, a);
    return hipGetLastError();
}

// J from the deterministic integer accumulators, which are cleared for the
// next step.
__global__ void __launch_bounds__(256) j_from_fixed_kernel(int64_t n, DetJ det, double* J0,
                                                           double* J1, double* J2) {
#pragma clang fp contract(off)
    const double s_hi = 1.0 / det.scale;
    const double s_lo = s_hi / (double)(1 << kDetLoBits);
    double* const J[3] = {J0, J1, J2};
    for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const long long h = (long long)det.hi[c][i];
            const long long l = det.lo[c][i];
            J[c][i] = (double)h * s_hi + (double)l * s_lo;
            det.hi[c][i] = 0ull;
            det.lo[c][i] = 0ll;
        }
    }
}

hipError_t launch_j_from_fixed(int64_t n, const DetJ& det, double* const J[3], hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    hipLaunchKernelGGL(j_from_fixed_kernel, dim3((int)b), dim3(256), 0, s, n, det, J[0], J[1],
                       J[2]);
    return hipGetLastError();
}

hipError_t launch_zero(double* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace pic
