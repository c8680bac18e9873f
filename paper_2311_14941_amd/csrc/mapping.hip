// Zonal reference-cell mapping (paper Sec. 2.5: the load-balanced solver
// the paper adopts maps the chemistry of low-reactivity regions from a
// reference cell instead of integrating every cell).  Around one
// integration launch:
//   1. classify: per cell, Bilger's coupling function beta = sum_k w_k Y_k,
//      the mixture fraction Z = (beta - beta_ox) / (beta_fuel - beta_ox);
//      a cell with finite inputs, T, p, dt > 0 and Z < z_tol falls in the
//      zone of its temperature band (and pressure band) and claims the zone
//      with an atomic minimum of its index;
//   2. assign: ref[c] = the zone's lowest-index cell (c itself when not
//      mappable); cells whose ref is another cell are skipped by the
//      integration kernels;
//   3. apply: each mapped cell takes its reference's change scaled by the
//      ratio of the steps, y1 = y0 + (y1_ref - y0_ref) dt / dt_ref, the
//      reference's status and zero step counts.
// One thread per cell; species rows are read with unit stride across the
// threads of a block (the SoA state layout), so every pass is a few
// coalesced sweeps over the batch, bound by HBM bandwidth.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>

#include "devmech.hpp"

namespace scdev {

constexpr int MAP_BLOCK = 256;

__global__ void __launch_bounds__(MAP_BLOCK) k_map_clear(int32_t *table, int64_t nz)
{
    const int64_t i = (int64_t)blockIdx.x * MAP_BLOCK + threadIdx.x;
    if (i < nz) table[i] = INT_MAX;
}

// zone of cell c, or -1 when it is not mappable
__device__ __forceinline__ int cell_zone(const MapParams &mp, int N, int64_t c, const double *T, const double *p,
                                         const double *Y, int64_t ld, const double *dt)
{
    // beta summed species by species, each product rounded before the sum
    double beta = 0.0;
    for (int k = 0; k < N; ++k) beta = __dadd_rn(beta, __dmul_rn(mp.w[k], Y[(int64_t)k * ld + c]));
    const double Z = (beta - mp.beta_ox) / mp.dbeta;
    const double Tc = T[c], pc = p[c], dtc = dt[c];
    if (!(isfinite(Z) && isfinite(Tc) && isfinite(pc) && isfinite(dtc))) return -1;
    if (!(Tc > 0.0 && pc > 0.0 && dtc > 0.0 && Z < mp.z_tol)) return -1;
    const double bT = floor(Tc / mp.dT);
    if (!(bT < (double)mp.nT)) return -1;
    int ip = 0;
    if (mp.dlnp > 0.0) {
        const double bp = floor(log(pc) / mp.dlnp);
        if (!(bp >= 0.0 && bp < (double)mp.np)) return -1;
        ip = (int)bp;
    }
    return (int)bT + mp.nT * ip;
}

__global__ void __launch_bounds__(MAP_BLOCK) k_map_zone(MapParams mp, int N, int64_t n, const double *T,
                                                        const double *p, const double *Y, int64_t ld,
                                                        const double *dt, int32_t *ref)
{
    const int64_t c = (int64_t)blockIdx.x * MAP_BLOCK + threadIdx.x;
    if (c >= n) return;
    const int z = cell_zone(mp, N, c, T, p, Y, ld, dt);
    ref[c] = z;  // the zone, until the assignment pass
    if (z >= 0) atomicMin(&mp.table[z], (int32_t)c);
}

__global__ void __launch_bounds__(MAP_BLOCK) k_map_assign(const int32_t *table, int64_t n, int32_t *ref)
{
    const int64_t c = (int64_t)blockIdx.x * MAP_BLOCK + threadIdx.x;
    if (c >= n) return;
    const int z = ref[c];
    ref[c] = z >= 0 ? table[z] : (int32_t)c;
}

__global__ void __launch_bounds__(MAP_BLOCK) k_map_apply(int N, int64_t n, const int32_t *ref, const double *T0,
                                                         const double *Y0, int64_t ld, const double *dt, double *T1,
                                                         double *Y1, int32_t *st, int32_t *na, int32_t *nr)
{
    const int64_t c = (int64_t)blockIdx.x * MAP_BLOCK + threadIdx.x;
    if (c >= n) return;
    const int64_t r = ref[c];
    if (r == c) return;
    const double s = dt[c] / dt[r];
    T1[c] = T0[c] + (T1[r] - T0[r]) * s;
    for (int k = 0; k < N; ++k) {
        const int64_t o = (int64_t)k * ld;
        Y1[o + c] = Y0[o + c] + (Y1[o + r] - Y0[o + r]) * s;
    }
    st[c] = st[r];
    if (na) na[c] = 0;
    if (nr) nr[c] = 0;
}

static unsigned blocks(int64_t n) { return (unsigned)((n + MAP_BLOCK - 1) / MAP_BLOCK); }

hipError_t launch_map_classify(const MapParams &mp, int N, int64_t n, const double *T, const double *p,
                               const double *Y, int64_t ld, const double *dt, int32_t *ref, hipStream_t s)
{
    const int64_t nz = (int64_t)mp.nT * mp.np;
    hipLaunchKernelGGL(k_map_clear, dim3(blocks(nz)), dim3(MAP_BLOCK), 0, s, mp.table, nz);
    hipLaunchKernelGGL(k_map_zone, dim3(blocks(n)), dim3(MAP_BLOCK), 0, s, mp, N, n, T, p, Y, ld, dt, ref);
    hipLaunchKernelGGL(k_map_assign, dim3(blocks(n)), dim3(MAP_BLOCK), 0, s, (const int32_t *)mp.table, n, ref);
    return hipGetLastError();
}

hipError_t launch_map_apply(int N, int64_t n, const int32_t *ref, const double *T0, const double *Y0, int64_t ld,
                            const double *dt, double *T1, double *Y1, int32_t *st, int32_t *na, int32_t *nr,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_map_apply, dim3(blocks(n)), dim3(MAP_BLOCK), 0, s, N, n, ref, T0, Y0, ld, dt, T1, Y1, st,
                       na, nr);
    return hipGetLastError();
}

}  // namespace scdev
