// Device view of a compiled mechanism and the launch interface of the
// kernels (shared by kernels.hip and capi.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "mech.hpp"
#include "stiffchem.h"

namespace scdev {

// One reaction's parameters, read by the lane that handles the reaction
// (160 bytes; the 64 lanes of a pass read 64 consecutive records).  Records
// are in the compiler's execution order (by kind, then side sizes).
struct RxRec {
    double lnA, b, EaR;            // SI ln A (incl. the cgs conversion), b, Ea/R
    double eam1[sc::MAXENH];       // alpha - 1 of the enhanced third-body species
    int32_t kind, nr, np, dnu, neff, tix;
    int32_t rsp[sc::MAXSIDE], rnu[sc::MAXSIDE], psp[sc::MAXSIDE], pnu[sc::MAXSIDE];
    int32_t esp[sc::MAXENH];
    int32_t orig;  // index of the reaction in the mechanism text (for dlnA)
    int32_t pad[3];
};
static_assert(sizeof(RxRec) % 16 == 0, "record size");

struct TroeRec {
    double lnA0, b0, Ea0R, a, iT3, iT1, T2, pad;
};

// A compiled mechanism on the device: species table sp = W[N] invW[N]
// nasa[7][N] (species index fastest), one record per reaction and per Troe
// reaction.  Three base pointers keep the kernels' scalar-register footprint
// small.
struct DevMech {
    int N, R, nt;
    int cv;  // 1: constant-volume reactor (the per-cell p input is the density)
    double Rgas, lnp0R;  // lnp0R = ln(p0 / Rgas)
    const double *sp;
    const RxRec *rx;
    const TroeRec *troe;

    __host__ __device__ const double *W() const { return sp; }
    __host__ __device__ const double *invW() const { return sp + N; }
    __host__ __device__ const double *nasa() const { return sp + 2 * N; }  // [c*N + k]
};

// The sparse kernels' view of a mechanism's compiled sparse algebra (device
// pointers) and their per-cell LDS layout (offsets in doubles; NV = 64 VPL
// doubles per state vector).
struct DevSparse {
    int n, nnz, nl_lu, nl_fw, nl_bw, n_u;
    int E, C, G, H, WD, UA, U, X, DINV, size;  // LDS offsets of one cell's region and its size (doubles)
    int NV;   // vector stride: lanes per cell times slots per lane
    int cpw;  // cells per wave (1, 2 or 4): each cell takes 64 / cpw lanes
    int tail0;  // first position of the dense trailing block (factorised in registers)
    const int *lu_b_lvl, *lu_c_lvl, *fw_lvl, *bw_lvl;
    const uint64_t *lu_b;  // widened to the c items' width: e_ik | e_kk << 16
    const uint32_t *lu_u, *diag;
    const uint64_t *lu_c, *fw, *bw;
    const uint16_t *rxi;   // [R][RXI_SIZE], reaction execution order
    const int32_t *comp;   // per species k: pos, e_kk, e_kT, e_kS, e_Tk, e_Sk; then pos_T, e_TT, e_SS
    const uint16_t *emap;    // n * n: (row, column) position -> entry or NOENT, row-major
    const int32_t *cstart;   // n + 1: first entry of each column (entries are numbered column by column)
    const uint64_t *cmask;   // 2 n: rows with an entry in column k, lanes 0-63 then 64-127
    const uint32_t *swf, *swb;  // n <= 64: per column the strictly lower (upper) rows' mask and first entry
    const uint16_t *swfi, *swbi;  // n <= 64: per column and row the lower (upper) entry, or nnz (zero slot)
    // interpolated thermodynamics (null: exact): per interval of ln T and
    // reaction (execution order) the 2 (ideg + 1) coefficients of -dG/RT and
    // dH/RT in t = 2 (ln T - u_i) iinvdu - 1
    const double *itab;
    int ideg, inint;
    double iu0, iinvdu;
};
constexpr int CMP = 6;  // comp entries per species

struct Opts {
    double rtol, atol;
    double hmax_frac;  // > 0: steps capped at hmax_frac * dt
    int max_steps;
    int fixed;  // 1: fixed steps of the caller's h, no error control
};

hipError_t launch_rhs(int np, const DevMech &m, int64_t n, const double *T, const double *p, const double *Y,
                      int64_t ld, const double *dlnA, double *fT, double *fY, hipStream_t s);
hipError_t launch_jac(int np, const DevMech &m, int64_t n, const double *T, const double *p, const double *Y,
                      int64_t ld, const double *dlnA, double *J, hipStream_t s);
hipError_t launch_linsolve(int np, const DevMech &m, int64_t n, const double *T, const double *p,
                           const double *Y, int64_t ld, const double *dlnA, const double *hg, const double *b,
                           double *x, hipStream_t s);
hipError_t launch_integrate(int np, const DevMech &m, const Opts &o, int method, int64_t n,
                            const double *T0, const double *p, const double *Y0, int64_t ld, const double *dt,
                            const double *dlnA, double *h_io, double *T1, double *Y1, int32_t *st, int32_t *na,
                            int32_t *nr, const int32_t *ref, hipStream_t s);
hipError_t launch_integrate_persistent(int np, const DevMech &m, const Opts &o, int method, int64_t n,
                                       const double *T0, const double *p, const double *Y0, int64_t ld,
                                       const double *dt, const double *dlnA, double *h_io, double *T1, double *Y1,
                                       int32_t *st, int32_t *na, int32_t *nr, unsigned long long *queue,
                                       const int32_t *perm, int tile, int grid, const int32_t *ref, hipStream_t s);
hipError_t launch_integrate_static(int np, const DevMech &m, const Opts &o, int method, int64_t n,
                                   const double *T0, const double *p, const double *Y0, int64_t ld, const double *dt,
                                   const double *dlnA, double *h_io, double *T1, double *Y1, int32_t *st,
                                   int32_t *na, int32_t *nr, int grid, const int32_t *ref, hipStream_t s);
hipError_t order_cells(int order, int64_t n, const double *dt, const int32_t *na, const int32_t *nr,
                       void **ws, size_t *ws_bytes, int32_t **perm, hipStream_t s);
hipError_t order_ws_need(int order, int64_t n, size_t *need, hipStream_t s);
hipError_t order_cells_in(int order, int64_t n, const double *dt, const int32_t *na, const int32_t *nr, void *ws,
                          size_t ws_bytes, int32_t **perm, hipStream_t s);
// device address, size and cell limit of the allocation-free entry point's
// fixed scratch on `device` (which must be current)
hipError_t noalloc_scratch(int device, void **ptr, size_t *bytes, int64_t *max_cells);
hipError_t launch_zero_u64(unsigned long long *p, hipStream_t s);
int persistent_capacity(int np, int device);

// sparse linear algebra kernels (sparse.hip); vpl = state components per lane
hipError_t launch_rhs_sp(int vpl, const DevMech &m, const DevSparse &sp, int64_t n, const double *T,
                         const double *p, const double *Y, int64_t ld, const double *dlnA, double *fT, double *fY,
                         hipStream_t s);
hipError_t launch_jac_sp(int vpl, const DevMech &m, const DevSparse &sp, int64_t n, const double *T,
                         const double *p, const double *Y, int64_t ld, const double *dlnA, double *J,
                         hipStream_t s);
hipError_t launch_linsolve_sp(int vpl, const DevMech &m, const DevSparse &sp, int64_t n, const double *T,
                              const double *p, const double *Y, int64_t ld, const double *dlnA, const double *hg,
                              const double *b, double *x, hipStream_t s);
hipError_t launch_integrate_sp(int vpl, const DevMech &m, const DevSparse &sp, const Opts &o, int64_t n,
                               const double *T0, const double *p, const double *Y0, int64_t ld, const double *dt,
                               const double *dlnA, double *h_io, double *T1, double *Y1, int32_t *st, int32_t *na,
                               int32_t *nr, const int32_t *ref, hipStream_t s);
hipError_t launch_integrate_sp_persistent(int vpl, const DevMech &m, const DevSparse &sp, const Opts &o,
                                          int64_t n, const double *T0, const double *p, const double *Y0,
                                          int64_t ld, const double *dt, const double *dlnA, double *h_io,
                                          double *T1, double *Y1, int32_t *st, int32_t *na, int32_t *nr,
                                          unsigned long long *queue, const int32_t *perm, int tile, int grid,
                                          const int32_t *ref, hipStream_t s);
hipError_t launch_integrate_sp_static(int vpl, const DevMech &m, const DevSparse &sp, const Opts &o, int64_t n,
                                      const double *T0, const double *p, const double *Y0, int64_t ld,
                                      const double *dt, const double *dlnA, double *h_io, double *T1, double *Y1,
                                      int32_t *st, int32_t *na, int32_t *nr, int grid, const int32_t *ref,
                                      hipStream_t s);
int persistent_capacity_sp(int vpl, const DevSparse &sp, int device);

// zonal reference-cell mapping (mapping.hip): the zone table is cleared,
// every mappable cell claims its zone (lowest index wins) and gets its
// reference in ref (ref[c] = c for cells that are integrated); after the
// integration, apply writes the mapped cells from their references
struct MapParams {
    const double *w;     // N per-species weights of Bilger's coupling function
    double beta_ox, dbeta, z_tol;  // dbeta = beta_fuel - beta_ox
    double dT, dlnp;     // band widths (dlnp = 0: no pressure bands)
    int nT, np;          // band counts; the table holds nT * np zones
    int32_t *table;      // nT * np zone claims
};
hipError_t launch_map_classify(const MapParams &mp, int N, int64_t n, const double *T, const double *p,
                               const double *Y, int64_t ld, const double *dt, int32_t *ref, hipStream_t s);
hipError_t launch_map_apply(int N, int64_t n, const int32_t *ref, const double *T0, const double *Y0, int64_t ld,
                            const double *dt, double *T1, double *Y1, int32_t *st, int32_t *na, int32_t *nr,
                            hipStream_t s);

// adjoint (adjoint.hip)
hipError_t launch_vjp(int np, const DevMech &m, int64_t n, const double *T, const double *p, const double *Y,
                      int64_t ld, const double *dlnA, const double *wT, const double *wY, double *gT, double *gY,
                      double *gcell, hipStream_t s);
hipError_t launch_adjoint(int np, const DevMech &m, const Opts &o, int64_t n, const double *T0, const double *p,
                          const double *Y0, int64_t ld, const double *dt, const double *dlnA, const double *h_in,
                          const double *gT1, const double *gY1, double *gT0, double *gY0, double *gcell,
                          int32_t *st, int32_t *na, double *T1, double *Y1, double *scratch, int64_t slot_doubles,
                          int hcap, unsigned long long *queue, const int32_t *perm, int grid, hipStream_t s);
hipError_t launch_sum_cells(const double *g, int64_t n, int R, double *out, hipStream_t s);
int adjoint_capacity(int np, int R, int device);

// operator-split driver support (transport.hip)
hipError_t launch_transport2d(int nx, int ny, int ncomp, const double *in, int64_t ld, const double *u,
                              const double *dt, double dx, double D, const double *inflow, double *out,
                              hipStream_t s);
int adjoint_slot_checkpoints();
size_t lds_bytes_for(int np);

}  // namespace scdev
