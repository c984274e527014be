// Maxwell integration on the Yee lattice (stage 1 of the PIC step of
// arXiv:1608.01009, Section 2), with B kept at integer time levels:
//   B <- B - dt/2 curl E;  E <- E + dt (curl B - J);  B <- B - dt/2 curl E.
// Three stencil passes over the periodic grid (each reads the neighbours the
// previous pass wrote).  The E pass also clears the J buffer that the next
// step deposits into.  The stencils are written in the order of the textbook
// differences with contraction off, so E and B are reproducible bit for bit
// given the same J.
#include "pic_internal.h"

namespace pic {
namespace {

constexpr int kBlock = 256;

struct FArgs {
    int n[3];
    int ncell;
    double dt, hdt;
    double dx[3];
    double* E[3];
    double* B[3];
    const double* J[3];
    double* Jc[3];
};

__global__ void __launch_bounds__(kBlock) half_b_kernel(const FArgs a) {
#pragma clang fp contract(off)
    const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
    for (int c = blockIdx.x * kBlock + threadIdx.x; c < a.ncell; c += gridDim.x * kBlock) {
        const int i = c % nx;
        const int jk = c / nx;
        const int j = jk % ny, k = jk / ny;
        const int ip = (i + 1 == nx) ? c - i : c + 1;
        const int jp = (j + 1 == ny) ? c - j * nx : c + nx;
        const int kp = (k + 1 == nz) ? c - k * nx * ny : c + nx * ny;
        const double ex = a.E[0][c], ey = a.E[1][c], ez = a.E[2][c];
        const double cx = (a.E[2][jp] - ez) / a.dx[1] - (a.E[1][kp] - ey) / a.dx[2];
        const double cy = (a.E[0][kp] - ex) / a.dx[2] - (a.E[2][ip] - ez) / a.dx[0];
        const double cz = (a.E[1][ip] - ey) / a.dx[0] - (a.E[0][jp] - ex) / a.dx[1];
        a.B[0][c] = a.B[0][c] - a.hdt * cx;
        a.B[1][c] = a.B[1][c] - a.hdt * cy;
        a.B[2][c] = a.B[2][c] - a.hdt * cz;
    }
}

__global__ void __launch_bounds__(kBlock) full_e_kernel(const FArgs a) {
#pragma clang fp contract(off)
    const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
    for (int c = blockIdx.x * kBlock + threadIdx.x; c < a.ncell; c += gridDim.x * kBlock) {
        const int i = c % nx;
        const int jk = c / nx;
        const int j = jk % ny, k = jk / ny;
        const int im = (i == 0) ? c + nx - 1 : c - 1;
        const int jm = (j == 0) ? c + (ny - 1) * nx : c - nx;
        const int km = (k == 0) ? c + (nz - 1) * nx * ny : c - nx * ny;
        const double bx = a.B[0][c], by = a.B[1][c], bz = a.B[2][c];
        const double cx = (bz - a.B[2][jm]) / a.dx[1] - (by - a.B[1][km]) / a.dx[2];
        const double cy = (bx - a.B[0][km]) / a.dx[2] - (bz - a.B[2][im]) / a.dx[0];
        const double cz = (by - a.B[1][im]) / a.dx[0] - (bx - a.B[0][jm]) / a.dx[1];
        a.E[0][c] = a.E[0][c] + a.dt * (cx - a.J[0][c]);
        a.E[1][c] = a.E[1][c] + a.dt * (cy - a.J[1][c]);
        a.E[2][c] = a.E[2][c] + a.dt * (cz - a.J[2][c]);
        a.Jc[0][c] = 0.0;
        a.Jc[1][c] = 0.0;
        a.Jc[2][c] = 0.0;
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

hipError_t launch_fdtd(const Geom& g, const Fields& f, double* const J[3],
                       double* const Jclear[3], hipStream_t s) {
    FArgs a;
    for (int d = 0; d < 3; ++d) {
        a.n[d] = g.n[d];
        a.dx[d] = g.dx[d];
        a.E[d] = f.E[d];
        a.B[d] = f.B[d];
        a.J[d] = J[d];
        a.Jc[d] = Jclear[d];
    }
    a.ncell = g.ncell;
    a.dt = g.dt;
    a.hdt = 0.5 * g.dt;
    const int nb = grid_for(g.ncell);
    hipLaunchKernelGGL(half_b_kernel, dim3(nb), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(full_e_kernel, dim3(nb), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(half_b_kernel, dim3(nb), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_zero(double* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace pic
