// Transport step of the operator-split driver: explicit first-order upwind
// advection along x plus diffusion on a uniform 2-D grid, every cell with
// its own (local) time step.  This is the cheap mixing operator that sits
// between chemistry substeps (paper Sec. 2.5: chemistry per cell, local time
// stepping); it is not part of the chemistry integration.
//
// With u >= 0, Co = u dt/dx, Fo = D dt/dx^2 and Co + 4 Fo <= 1 the update
//   q' = q - Co (q - q_W) + Fo (q_E + q_W + q_N + q_S - 4 q)
// is a convex combination of neighbouring values, so mass fractions stay in
// [0, 1] and keep summing to one.  Boundaries: x = 0 takes the inflow
// profile (Dirichlet), the other three are zero-gradient.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace scdev {

// one thread per (cell, component); components are species-major rows of
// ld values (the library's state layout), cells row-major c = iy*nx + ix
__global__ void __launch_bounds__(256) k_transport2d(int nx, int ny, int ncomp, const double *in, int64_t ld,
                                                     const double *u, const double *dt, double dx, double D,
                                                     const double *inflow, double *out)
{
    const int64_t n = (int64_t)nx * ny;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * ncomp) return;
    const int k = (int)(t / n);
    const int64_t c = t - (int64_t)k * n;
    const int iy = (int)(c / nx), ix = (int)(c - (int64_t)iy * nx);
    const double *q = in + (int64_t)k * ld;
    const double qc = q[c];
    const double qw = ix > 0 ? q[c - 1] : inflow[(int64_t)k * ny + iy];
    const double qe = ix < nx - 1 ? q[c + 1] : qc;
    const double qs = iy > 0 ? q[c - nx] : qc;
    const double qn = iy < ny - 1 ? q[c + nx] : qc;
    const double co = u[c] * dt[c] / dx;
    const double fo = D * dt[c] / (dx * dx);
    out[(int64_t)k * ld + c] = qc - co * (qc - qw) + fo * (qe + qw + qn + qs - 4.0 * qc);
}

hipError_t launch_transport2d(int nx, int ny, int ncomp, const double *in, int64_t ld, const double *u,
                              const double *dt, double dx, double D, const double *inflow, double *out,
                              hipStream_t s)
{
    const int64_t total = (int64_t)nx * ny * ncomp;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL(k_transport2d, dim3(blocks), dim3(256), 0, s, nx, ny, ncomp, in, ld, u, dt, dx, D, inflow,
                       out);
    return hipGetLastError();
}

}  // namespace scdev
