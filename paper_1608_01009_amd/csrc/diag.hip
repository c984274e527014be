// Diagnostics of the PIC state (not on the timed path): field and kinetic
// energies, cloud-in-cell charge density at the nodes, the Gauss residual
// div E - rho and div B.  Sums use per-block reductions and FP64 global
// atomics (their order is unspecified; these are reported values, not state).
#include "pic_internal.h"

namespace pic {
namespace {

constexpr int kBlock = 256;

__device__ double block_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__device__ double block_max(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kBlock) sumsq_kernel(const double* a, const double* b,
                                                       const double* c, int64_t n, double* acc) {
    __shared__ double red[kBlock];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        s += a[i] * a[i] + b[i] * b[i] + c[i] * c[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) unsafeAtomicAdd(acc, s);
}

__global__ void __launch_bounds__(kBlock) kinetic_kernel(const double* ux, const double* uy,
                                                         const double* uz, int64_t n,
                                                         double* acc, const double* x,
                                                         double* cnt) {
    __shared__ double red[kBlock];
    double s = 0.0, live = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        if (x && x[i] < 0.0) continue;       // removed (absorbing x)
        // gamma - 1 without the cancellation of sqrt(1 + u^2) - 1 at small u
        const double u2 = (ux[i] * ux[i] + uy[i] * uy[i]) + uz[i] * uz[i];
        s += u2 / (1.0 + sqrt(1.0 + u2));
        live += 1.0;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) unsafeAtomicAdd(acc, s);
    if (cnt) {
        __syncthreads();
        live = block_sum(live, red);
        if (threadIdx.x == 0) unsafeAtomicAdd(cnt, live);
    }
}

__device__ __forceinline__ int wrapi(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

__global__ void __launch_bounds__(kBlock) rho_kernel(Geom g, double qv, const double* x,
                                                     const double* y, const double* z, int64_t n,
                                                     double* rho) {
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    for (int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * kBlock) {
        const double xp[3] = {x[p], y[p], z[p]};
        if (xp[0] < 0.0) continue;             // removed (absorbing x)
        int i[3];
        double f[3];
        for (int d = 0; d < 3; ++d) {
            const double fl = floor(xp[d]);
            i[d] = (int)fl;
            f[d] = xp[d] - fl;
        }
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int c = 0; c < 2; ++c) {
                    const double w = (a ? f[0] : 1.0 - f[0]) * (b ? f[1] : 1.0 - f[1]) *
                                     (c ? f[2] : 1.0 - f[2]);
                    unsafeAtomicAdd(&rho[wrapi(i[0] + a, nx) +
                                         nx * (wrapi(i[1] + b, ny) + ny * wrapi(i[2] + c, nz))],
                                    qv * w);
                }
    }
}

__global__ void __launch_bounds__(kBlock) gauss_kernel(Geom g, const double* ex, const double* ey,
                                                       const double* ez, const double* rho,
                                                       double* out) {
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    for (int c = blockIdx.x * kBlock + threadIdx.x; c < g.ncell; c += gridDim.x * kBlock) {
        const int i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
        const int im = (i == 0) ? c + nx - 1 : c - 1;
        const int jm = (j == 0) ? c + (ny - 1) * nx : c - nx;
        const int km = (k == 0) ? c + (nz - 1) * nx * ny : c - nx * ny;
        out[c] = ((ex[c] - ex[im]) / g.dx[0] + (ey[c] - ey[jm]) / g.dx[1] +
                  (ez[c] - ez[km]) / g.dx[2]) - rho[c];
        // absorbing x: the Mur planes do not follow Gauss's law
        if (g.absorb_x && (i == 0 || i == nx - 1)) out[c] = 0.0;
    }
}

__global__ void __launch_bounds__(kBlock) divb_kernel(Geom g, const double* bx, const double* by,
                                                      const double* bz, double* out) {
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    for (int c = blockIdx.x * kBlock + threadIdx.x; c < g.ncell; c += gridDim.x * kBlock) {
        const int i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
        const int ip = (i + 1 == nx) ? c - i : c + 1;
        const int jp = (j + 1 == ny) ? c - j * nx : c + nx;
        const int kp = (k + 1 == nz) ? c - k * nx * ny : c + nx * ny;
        out[c] = (bx[ip] - bx[c]) / g.dx[0] + (by[jp] - by[c]) / g.dx[1] +
                 (bz[kp] - bz[c]) / g.dx[2];
        if (g.absorb_x && i == nx - 1) out[c] = 0.0;   // the cell outside the box
    }
}

__global__ void __launch_bounds__(kBlock) maxabs_kernel(const double* a, const double* b, int64_t n,
                                                        unsigned long long* acc) {
    __shared__ double red[kBlock];
    double m = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        m = fmax(m, fabs(a[i] - b[i]));
    m = block_max(m, red);
    // non-negative doubles order like their bit patterns
    if (threadIdx.x == 0) atomicMax(acc, (unsigned long long)__double_as_longlong(m));
}

int grid_for(int64_t n) {
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b > 4096) b = 4096;
    return b < 1 ? 1 : (int)b;
}

}  // namespace

hipError_t launch_sum_squares(const double* const a[3], int64_t n, double* acc, hipStream_t s) {
    hipLaunchKernelGGL(sumsq_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, a[0], a[1], a[2], n,
                       acc);
    return hipGetLastError();
}

hipError_t launch_kinetic(const double* ux, const double* uy, const double* uz, int64_t n,
                          double* acc, hipStream_t s, const double* x, double* cnt) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(kinetic_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, ux, uy, uz, n, acc,
                       x, cnt);
    return hipGetLastError();
}

hipError_t launch_rho(const Geom& g, double qv, const double* x, const double* y,
                      const double* z, int64_t n, double* rho, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(rho_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, g, qv, x, y, z, n, rho);
    return hipGetLastError();
}

hipError_t launch_gauss(const Geom& g, const Fields& f, const double* rho, double* out,
                        hipStream_t s) {
    hipLaunchKernelGGL(gauss_kernel, dim3(grid_for(g.ncell)), dim3(kBlock), 0, s, g, f.E[0],
                       f.E[1], f.E[2], rho, out);
    return hipGetLastError();
}

hipError_t launch_divb(const Geom& g, const Fields& f, double* out, hipStream_t s) {
    hipLaunchKernelGGL(divb_kernel, dim3(grid_for(g.ncell)), dim3(kBlock), 0, s, g, f.B[0],
                       f.B[1], f.B[2], out);
    return hipGetLastError();
}

hipError_t launch_maxabs_diff(const double* a, const double* b, int64_t n,
                              unsigned long long* acc_bits, hipStream_t s) {
    hipLaunchKernelGGL(maxabs_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, a, b, n, acc_bits);
    return hipGetLastError();
}

}  // namespace pic
