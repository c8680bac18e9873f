// Forward kernels: right-hand side, Jacobian and linear-solve probes, and
// the batched integration in plain (one workgroup per cell), persistent
// (resident grid pulling cells from a queue) and static-mapping launches,
// plus the cell ordering for the queue.  Building blocks live in core.hpp.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include <hipcub/hipcub.hpp>

#include "core.hpp"

namespace scdev {

template <int NP, bool CV>
__global__ void __launch_bounds__(WAVE) k_rhs(DevMech mk, int64_t n, const double *T, const double *p,
                                              const double *Y, int64_t ld, const double *dlnA, double *fT,
                                              double *fY)
{
    extern __shared__ double lds[];
    const DevMech m = fix_reactor<CV>(mk);
    const int lane = threadIdx.x;
    const int64_t c = blockIdx.x;
    if (c >= n) return;
    const double y = load_state(m, T, Y, ld, c, lane);
    const double f = rhs<NP>(m, lds, y, p[c], dlnA, lane);
    if (lane < m.N) fY[(int64_t)lane * ld + c] = f;
    if (lane == m.N) fT[c] = f;
}

template <int NP, bool CV>
__global__ void __launch_bounds__(WAVE) k_jac(DevMech mk, int64_t n, const double *T, const double *p,
                                              const double *Y, int64_t ld, const double *dlnA, double *J)
{
    extern __shared__ double lds[];
    const DevMech m = fix_reactor<CV>(mk);
    const int lane = threadIdx.x;
    const int64_t c = blockIdx.x;
    if (c >= n) return;
    const double y = load_state(m, T, Y, ld, c, lane);
    RowCoef rc;
    rhs_jac<NP>(m, lds, y, p[c], dlnA, lane, rc);
    double a[NP];
    jac_row<NP>(m, lds, rc, lane, a);
    const int nn = m.N + 1;
    if (lane < nn) {
        double *out = J + (c * nn + lane) * nn;
#pragma unroll
        for (int k = 0; k < NP; ++k)
            if (k < nn) out[k] = a[k];
    }
}

template <int NP, bool CV>
__global__ void __launch_bounds__(WAVE) k_linsolve(DevMech mk, int64_t n, const double *T, const double *p,
                                                   const double *Y, int64_t ld, const double *dlnA,
                                                   const double *hg, const double *b, double *x)
{
    extern __shared__ double lds[];
    const DevMech m = fix_reactor<CV>(mk);
    const int lane = threadIdx.x;
    const int64_t c = blockIdx.x;
    if (c >= n) return;
    const double y = load_state(m, T, Y, ld, c, lane);
    RowCoef rc;
    rhs_jac<NP>(m, lds, y, p[c], dlnA, lane, rc);
    const double dinv = factor_matrix<NP>(m, lds, rc, lane, 1.0 / hg[c], lds + Lds<NP>::P);
    const int nn = m.N + 1;
    const double bb = lane < nn ? b[c * nn + lane] : 0.0;
    const double xx = lu_solve<NP>(lds + Lds<NP>::P, dinv, bb, lane);
    if (lane < nn) x[c * nn + lane] = xx;
}

// One cell over [0, dt] with the method METH and error control.
template <int NP, int METH>
__device__ void integrate_cell(const DevMech &m, const Opts &o, double *lds, int64_t c, int lane, const double *T0,
                               const double *P, const double *Y0, int64_t ld, const double *DT, const double *dlnA,
                               double *h_io, double *T1, double *Y1, int32_t *status, int32_t *nacc_out,
                               int32_t *nrej_out, const int32_t *ref)
{
    // a cell mapped onto another cell's result is left to the mapping pass
    if (ref && ref[c] != c) return;
    const int N = m.N;
    double y = load_state(m, T0, Y0, ld, c, lane);
    const double p = P[c], dt = DT[c];
    int st = SC_CELL_OK;
    Ctl s = ctl_init(initial_step(h_io, c, dt), dt);
    if (bad_input(m, y, p, dt, lane)) {
        st = SC_CELL_BAD_INPUT;
    } else if (dt > 0.0) {
        st = advance<NP, METH>(m, o, lds, y, p, dt, dlnA, lane, s);
    }
    if (lane < N) Y1[(int64_t)lane * ld + c] = y;
    if (lane == N) {
        T1[c] = y;
        status[c] = st;
        if (nacc_out) nacc_out[c] = s.nacc;
        if (nrej_out) nrej_out[c] = s.nrej;
        if (h_io && st == SC_CELL_OK && dt > 0.0) h_io[c] = s.hnext;
    }
}

template <int NP, bool CV, int METH>
__global__ void __launch_bounds__(WAVE) k_integrate(DevMech mk, Opts o, int64_t n, const double *T0, const double *P,
                                                    const double *Y0, int64_t ld, const double *DT,
                                                    const double *dlnA, double *h_io, double *T1, double *Y1,
                                                    int32_t *status, int32_t *nacc, int32_t *nrej,
                                                    const int32_t *ref)
{
    extern __shared__ double lds[];
    const DevMech m = fix_reactor<CV>(mk);
    const int64_t c = blockIdx.x;
    if (c >= n) return;
    integrate_cell<NP, METH>(m, o, lds, c, threadIdx.x, T0, P, Y0, ld, DT, dlnA, h_io, T1, Y1, status, nacc, nrej, ref);
}

// Persistent variant: a resident grid; each wave pulls tiles of `tile` cells
// from a global counter (optionally through a permutation, e.g. longest dt
// first) until the queue is drained.  Per-cell arithmetic is identical to the
// plain kernel, so results are bitwise equal.
template <int NP, bool CV, int METH>
__global__ void __launch_bounds__(WAVE) k_integrate_persistent(DevMech mk, Opts o, int64_t n, const double *T0,
                                                               const double *P, const double *Y0, int64_t ld,
                                                               const double *DT, const double *dlnA, double *h_io,
                                                               double *T1, double *Y1, int32_t *status,
                                                               int32_t *nacc, int32_t *nrej,
                                                               unsigned long long *queue, const int32_t *perm,
                                                               int tile, const int32_t *ref)
{
    extern __shared__ double lds[];
    const DevMech m = fix_reactor<CV>(mk);
    const int lane = threadIdx.x;
#pragma unroll 1
    while (true) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(queue, (unsigned long long)tile);
        base = __shfl(base, 0, WAVE);
        if (base >= (unsigned long long)n) break;
        const int64_t end = min((int64_t)base + tile, n);
#pragma unroll 1
        for (int64_t i = (int64_t)base; i < end; ++i) {
            const int64_t c = perm ? (int64_t)perm[i] : i;
            integrate_cell<NP, METH>(m, o, lds, c, lane, T0, P, Y0, ld, DT, dlnA, h_io, T1, Y1, status, nacc, nrej, ref);
        }
    }
}

// Static mapping (the baseline the queue is compared with): workgroup w owns
// cells [w*group, (w+1)*group) and integrates them one after another.
template <int NP, bool CV, int METH>
__global__ void __launch_bounds__(WAVE) k_integrate_static(DevMech mk, Opts o, int64_t n, const double *T0,
                                                           const double *P, const double *Y0, int64_t ld,
                                                           const double *DT, const double *dlnA, double *h_io,
                                                           double *T1, double *Y1, int32_t *status, int32_t *nacc,
                                                           int32_t *nrej, int64_t group, const int32_t *ref)
{
    extern __shared__ double lds[];
    const DevMech m = fix_reactor<CV>(mk);
    const int64_t c0 = (int64_t)blockIdx.x * group;
    const int64_t c1 = min(c0 + group, n);
#pragma unroll 1
    for (int64_t c = c0; c < c1; ++c)
        integrate_cell<NP, METH>(m, o, lds, c, threadIdx.x, T0, P, Y0, ld, DT, dlnA, h_io, T1, Y1, status, nacc, nrej, ref);
}

__global__ void k_zero_u64(unsigned long long *p) { *p = 0ull; }

__global__ void k_iota(int32_t *v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = (int32_t)i;
}

__global__ void k_cost(const int32_t *na, const int32_t *nr, int32_t *key, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) key[i] = na[i] + (nr ? nr[i] : 0);
}

// ---------------------------------------------------------------------------
// launchers (host)
// ---------------------------------------------------------------------------
template <int NP>
size_t lds_bytes() { return sizeof(double) * Lds<NP>::SIZE; }

// kernel variant by padded size and reactor model (m.cv); SC_KERNEL keeps
// the template argument list one macro argument of hipLaunchKernelGGL
#define SC_KERNEL(k) k<NPV, CVV>
#define SC_CASE(npv, ...)                                                             \
    case npv:                                                                         \
        if (m.cv) { constexpr int NPV = npv; constexpr bool CVV = true; __VA_ARGS__; } \
        else { constexpr int NPV = npv; constexpr bool CVV = false; __VA_ARGS__; }    \
        break;
// integration kernels: also by method (SC_METHOD_*)
#define SC_KERNEL_I(k) k<NPV, CVV, MV>
#define SC_CASE_I(npv, ...)                                                                              \
    case npv:                                                                                            \
        if (m.cv) {                                                                                      \
            constexpr int NPV = npv; constexpr bool CVV = true;                                          \
            if (method == SC_METHOD_EXTRAP) { constexpr int MV = SC_METHOD_EXTRAP; __VA_ARGS__; }       \
            else { constexpr int MV = SC_METHOD_ROS4; __VA_ARGS__; }                                     \
        } else {                                                                                         \
            constexpr int NPV = npv; constexpr bool CVV = false;                                         \
            if (method == SC_METHOD_EXTRAP) { constexpr int MV = SC_METHOD_EXTRAP; __VA_ARGS__; }       \
            else { constexpr int MV = SC_METHOD_ROS4; __VA_ARGS__; }                                     \
        }                                                                                                \
        break;
#define SC_DISPATCH_I(np, ...)                \
    switch (np) {                             \
    SC_CASE_I(16, __VA_ARGS__)                \
    SC_CASE_I(32, __VA_ARGS__)                \
    SC_CASE_I(56, __VA_ARGS__)                \
    SC_CASE_I(64, __VA_ARGS__)                \
    default: return hipErrorInvalidValue;     \
    }
#define SC_DISPATCH(np, ...)                  \
    switch (np) {                             \
    SC_CASE(16, __VA_ARGS__)                  \
    SC_CASE(32, __VA_ARGS__)                  \
    SC_CASE(56, __VA_ARGS__)                  \
    SC_CASE(64, __VA_ARGS__)                  \
    default: return hipErrorInvalidValue;     \
    }

hipError_t launch_rhs(int np, const DevMech &m, int64_t n, const double *T, const double *p, const double *Y,
                      int64_t ld, const double *dlnA, double *fT, double *fY, hipStream_t s)
{
    SC_DISPATCH(np, hipLaunchKernelGGL(SC_KERNEL(k_rhs), dim3((unsigned)n), dim3(WAVE), lds_bytes<NPV>(), s, m, n, T, p,
                                       Y, ld, dlnA, fT, fY));
    return hipGetLastError();
}

hipError_t launch_jac(int np, const DevMech &m, int64_t n, const double *T, const double *p, const double *Y,
                      int64_t ld, const double *dlnA, double *J, hipStream_t s)
{
    SC_DISPATCH(np, hipLaunchKernelGGL(SC_KERNEL(k_jac), dim3((unsigned)n), dim3(WAVE), lds_bytes<NPV>(), s, m, n, T, p,
                                       Y, ld, dlnA, J));
    return hipGetLastError();
}

hipError_t launch_linsolve(int np, const DevMech &m, int64_t n, const double *T, const double *p, const double *Y,
                           int64_t ld, const double *dlnA, const double *hg, const double *b, double *x,
                           hipStream_t s)
{
    SC_DISPATCH(np, hipLaunchKernelGGL(SC_KERNEL(k_linsolve), dim3((unsigned)n), dim3(WAVE), lds_bytes<NPV>(), s, m, n,
                                       T, p, Y, ld, dlnA, hg, b, x));
    return hipGetLastError();
}

hipError_t launch_integrate(int np, const DevMech &m, const Opts &o, int method, int64_t n, const double *T0,
                            const double *p, const double *Y0, int64_t ld, const double *dt, const double *dlnA,
                            double *h_io, double *T1, double *Y1, int32_t *st, int32_t *na, int32_t *nr,
                            const int32_t *ref, hipStream_t s)
{
    SC_DISPATCH_I(np, hipLaunchKernelGGL(SC_KERNEL_I(k_integrate), dim3((unsigned)n), dim3(WAVE), lds_bytes<NPV>(), s,
                                         m, o, n, T0, p, Y0, ld, dt, dlnA, h_io, T1, Y1, st, na, nr, ref));
    return hipGetLastError();
}

hipError_t launch_integrate_persistent(int np, const DevMech &m, const Opts &o, int method, int64_t n,
                                       const double *T0, const double *p, const double *Y0, int64_t ld,
                                       const double *dt, const double *dlnA, double *h_io, double *T1, double *Y1,
                                       int32_t *st, int32_t *na, int32_t *nr, unsigned long long *queue,
                                       const int32_t *perm, int tile, int grid, const int32_t *ref, hipStream_t s)
{
    SC_DISPATCH_I(np, hipLaunchKernelGGL(SC_KERNEL_I(k_integrate_persistent), dim3((unsigned)grid), dim3(WAVE),
                                         lds_bytes<NPV>(), s, m, o, n, T0, p, Y0, ld, dt, dlnA, h_io, T1, Y1, st, na,
                                         nr, queue, perm, tile, ref));
    return hipGetLastError();
}

hipError_t launch_integrate_static(int np, const DevMech &m, const Opts &o, int method, int64_t n,
                                   const double *T0, const double *p, const double *Y0, int64_t ld, const double *dt,
                                   const double *dlnA, double *h_io, double *T1, double *Y1, int32_t *st,
                                   int32_t *na, int32_t *nr, int grid, const int32_t *ref, hipStream_t s)
{
    const int64_t group = (n + grid - 1) / grid;
    const unsigned g = (unsigned)((n + group - 1) / group);
    SC_DISPATCH_I(np, hipLaunchKernelGGL(SC_KERNEL_I(k_integrate_static), dim3(g), dim3(WAVE), lds_bytes<NPV>(), s,
                                         m, o, n, T0, p, Y0, ld, dt, dlnA, h_io, T1, Y1, st, na, nr, group, ref));
    return hipGetLastError();
}

// Cell permutation for the persistent queue: indices sorted by descending
// key (dt, or the previous call's step count), by a device radix sort.
// Workspace layout: [perm_in | perm_out | keys_out | cost keys | temp].
namespace {
size_t up256(size_t b) { return (b + 255) / 256 * 256; }
}  // namespace

// Workspace bytes the ordering of n cells needs (a size query of the sort:
// no allocation, no launch).
hipError_t order_ws_need(int order, int64_t n, size_t *need, hipStream_t s)
{
    size_t tmp = 0;
    hipError_t e;
    if (order == SC_ORDER_DT)
        e = hipcub::DeviceRadixSort::SortPairsDescending(nullptr, tmp, (const double *)nullptr, (double *)nullptr,
                                                         (const int32_t *)nullptr, (int32_t *)nullptr, (int)n, 0, 64,
                                                         s);
    else
        e = hipcub::DeviceRadixSort::SortPairsDescending(nullptr, tmp, (const int32_t *)nullptr, (int32_t *)nullptr,
                                                         (const int32_t *)nullptr, (int32_t *)nullptr, (int)n, 0, 32,
                                                         s);
    if (e != hipSuccess) return e;
    *need = 2 * up256(sizeof(int32_t) * n) + 2 * up256(sizeof(double) * n) + up256(tmp);
    return hipSuccess;
}

// The ordering in a workspace the caller provides (at least order_ws_need
// bytes, 256-byte aligned); allocates nothing.
hipError_t order_cells_in(int order, int64_t n, const double *dt, const int32_t *na, const int32_t *nr, void *ws,
                          size_t ws_bytes, int32_t **perm, hipStream_t s)
{
    size_t need = 0;
    hipError_t e = order_ws_need(order, n, &need, s);
    if (e != hipSuccess) return e;
    if (ws_bytes < need) return hipErrorInvalidValue;
    const size_t b_perm = up256(sizeof(int32_t) * n), b_keys = up256(sizeof(double) * n);
    size_t tmp = need - 2 * b_perm - 2 * b_keys;
    char *base = (char *)ws;
    int32_t *pin = (int32_t *)base, *pout = (int32_t *)(base + b_perm);
    void *kout = base + 2 * b_perm, *kcost = base + 2 * b_perm + b_keys, *temp = base + 2 * b_perm + 2 * b_keys;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_iota, dim3(blocks), dim3(256), 0, s, pin, n);
    if (order == SC_ORDER_DT) {
        e = hipcub::DeviceRadixSort::SortPairsDescending(temp, tmp, dt, (double *)kout, pin, pout, (int)n, 0, 64, s);
    } else {
        hipLaunchKernelGGL(k_cost, dim3(blocks), dim3(256), 0, s, na, nr, (int32_t *)kcost, n);
        e = hipcub::DeviceRadixSort::SortPairsDescending(temp, tmp, (const int32_t *)kcost, (int32_t *)kout, pin, pout,
                                                         (int)n, 0, 32, s);
    }
    *perm = pout;
    return e != hipSuccess ? e : hipGetLastError();
}

// The ordering in a plan-owned workspace `ws`, grown on demand.
hipError_t order_cells(int order, int64_t n, const double *dt, const int32_t *na, const int32_t *nr,
                       void **ws, size_t *ws_bytes, int32_t **perm, hipStream_t s)
{
    size_t need = 0;
    hipError_t e = order_ws_need(order, n, &need, s);
    if (e != hipSuccess) return e;
    if (*ws_bytes < need) {
        if (*ws) (void)hipFree(*ws);
        *ws = nullptr;
        *ws_bytes = 0;
        if ((e = hipMalloc(ws, need)) != hipSuccess) return e;
        *ws_bytes = need;
    }
    return order_cells_in(order, n, dt, na, nr, *ws, *ws_bytes, perm, s);
}

// ---------------------------------------------------------------------------
// Fixed device scratch of the allocation-free integration entry point: the
// queue counter (first 256 bytes) and the cell-ordering workspace.  One copy
// per device, held until the process ends; every call on a device shares it
// (concurrent calls on one device race).  Host code reaches it only through
// the address hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)16 << 20;
constexpr int64_t NOALLOC_MAX_CELLS = 262144;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

// Resolve (once per device, with that device current) the device address of
// the scratch array.
hipError_t noalloc_scratch(int device, void **ptr, size_t *bytes, int64_t *max_cells)
{
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    *bytes = NOALLOC_SCRATCH_BYTES;
    *max_cells = NOALLOC_MAX_CELLS;
    return hipSuccess;
}

// clears the queue counter with a kernel (safe inside captured graphs)
hipError_t launch_zero_u64(unsigned long long *p, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, p);
    return hipGetLastError();
}

int persistent_capacity(int np, int device)
{
    int per_cu = 0, cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
    hipError_t e = hipErrorInvalidValue;
    switch (np) {
    case 16:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_integrate_persistent<16, false, SC_METHOD_ROS4>,
                                                         WAVE, lds_bytes<16>());
        break;
    case 32:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_integrate_persistent<32, false, SC_METHOD_ROS4>,
                                                         WAVE, lds_bytes<32>());
        break;
    case 56:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_integrate_persistent<56, false, SC_METHOD_ROS4>,
                                                         WAVE, lds_bytes<56>());
        break;
    case 64:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_integrate_persistent<64, false, SC_METHOD_ROS4>,
                                                         WAVE, lds_bytes<64>());
        break;
    default: break;
    }
    return e == hipSuccess ? per_cu * cus : 0;
}

size_t lds_bytes_for(int np)
{
    switch (np) {
    case 16: return lds_bytes<16>();
    case 32: return lds_bytes<32>();
    case 56: return lds_bytes<56>();
    case 64: return lds_bytes<64>();
    }
    return 0;
}

}  // namespace scdev
