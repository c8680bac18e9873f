/* stiffchem -- batched stiff chemistry integration on MI355X (gfx950).
 *
 * Every CFD cell is integrated as an independent homogeneous gas-phase
 * reactor (paper Sec. 1: one reactor per cell, cost proportional to the cell
 * count; Sec. 2.1, Eqs. 3-4: the species and heat source terms come from that
 * integration).  The reactor here is adiabatic, ideal-gas and at constant
 * pressure; its state is (T, Y_1..Y_N).  The integrator is a linearly implicit
 * (Rosenbrock) method fed by an analytical Jacobian (Sec. 2.5: sparse
 * analytical Jacobian, per-cell local time steps).
 *
 * Conventions for every call:
 *   - units are SI: T [K], p [Pa], Y [-], dt [s];
 *   - array arguments of sc_rhs, sc_jacobian, sc_linsolve, sc_integrate and
 *     sc_adjoint are DEVICE pointers on the plan's device, owned by the
 *     caller; mass fractions are species-major, Y[k * ld + c] for species k
 *     of cell c (ld >= n);
 *   - argument errors are returned synchronously, before any launch, with a
 *     message from sc_last_error(); device work is asynchronous on the given
 *     HIP stream (NULL = the default stream) and the caller synchronises;
 *   - per-cell failures never fail a call: they set the cell's status code;
 *   - no C++ exception or abort crosses this interface.
 * The library owns only sc_mech, sc_plan and its internal workspace.
 */
#ifndef STIFFCHEM_H
#define STIFFCHEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SC_OK = 0,
    SC_EINVAL = -1,       /* bad argument (NULL pointer, negative size, ...) */
    SC_EPARSE = -2,       /* malformed or inconsistent mechanism text */
    SC_ENOMEM = -3,       /* device or host allocation failed */
    SC_EHIP = -4,         /* a HIP runtime call failed */
    SC_EUNSUPPORTED = -5, /* mechanism larger than the kernels support */
    SC_EBUDGET = -6       /* adjoint checkpoints exceed the memory budget */
} sc_status;

/* per-cell status codes written by sc_integrate / sc_adjoint */
enum {
    SC_CELL_OK = 0,
    SC_CELL_MAX_STEPS = 1,   /* max_steps reached before t = dt */
    SC_CELL_H_UNDERFLOW = 2, /* step size fell below 1e-20 dt */
    SC_CELL_NONFINITE = 3,   /* five consecutive non-finite error estimates */
    SC_CELL_BAD_INPUT = 4    /* non-finite or non-positive T, p; dt < 0; non-finite Y */
};

/* integration modes */
enum {
    SC_MODE_PLAIN = 0,      /* one workgroup per cell, grid = cells */
    SC_MODE_PERSISTENT = 1, /* resident grid pulling cell tiles from a queue */
    SC_MODE_STATIC = 2      /* resident grid, workgroup w owns a fixed contiguous
                               group of cells (the static-mapping baseline) */
};

/* persistent-mode cell order */
enum {
    SC_ORDER_NONE = 0,     /* cells in index order */
    SC_ORDER_DT = 1,       /* longest dt first */
    SC_ORDER_COST = 2      /* most steps first, by the incoming n_acc + n_rej
                              (the previous call's counts: measured cost) */
};

typedef struct sc_mech sc_mech; /* immutable after load; shareable across threads */
typedef struct sc_plan sc_plan; /* a mechanism on one device; one stream at a time */

/* Reactor model of every cell (both adiabatic, ideal gas).  Constant
 * pressure: the per-cell array p of the calls below is the pressure [Pa],
 * energy balance on enthalpy.  Constant volume (a rigid vessel): that array
 * is the density rho [kg/m^3], held fixed while the pressure follows
 * p = rho R T / Wbar; energy balance on internal energy,
 *   dT/dt = -sum_k (h_k - R T) wdot_k / (rho cv),  cv = cp - R / Wbar,
 * and C_k = rho Y_k / W_k.  sc_vjp and sc_adjoint support constant
 * pressure only (SC_EUNSUPPORTED otherwise). */
typedef enum {
    SC_REACTOR_CONST_P = 0,
    SC_REACTOR_CONST_V = 1
} sc_reactor;

/* Integration method of sc_integrate.  ROS4: the 4-stage, order-4
 * L-stable Rosenbrock method with an embedded order-3 estimate (one
 * Jacobian, one factorisation and three right-hand sides per step).
 * EXTRAP: a standard extrapolation baseline, the linearly implicit Euler
 * method on the step-number sequence 1, 2, 3, 4 with Aitken-Neville
 * extrapolation to order 4, error from the order-3 entry (four
 * factorisations, ten substeps per step).  Both use the same analytical
 * Jacobian and step controller; sc_adjoint supports ROS4 only. */
typedef enum {
    SC_METHOD_ROS4 = 0,
    SC_METHOD_EXTRAP = 1
} sc_method;

/* Linear algebra of the implicit stages (paper Sec. 2.5: sparse analytical
 * Jacobian and sparse algebra management of the mechanism).  DENSE: the
 * (N+1)-square iteration matrix in registers, one row per lane, factorised
 * in natural order (N <= 63).  SPARSE: the bordered system of order N+2
 * (species block with its fixed sparsity, then the temperature and density
 * borders) in LDS, factorised in the mechanism compiler's minimum-degree
 * order by its static level schedule (N <= 127).  AUTO: dense where it
 * applies, else sparse. */
typedef enum {
    SC_LINALG_AUTO = 0,
    SC_LINALG_DENSE = 1,
    SC_LINALG_SPARSE = 2
} sc_linalg;

typedef struct {
    double rtol;        /* relative tolerance (default 1e-6) */
    double atol;        /* absolute tolerance, every component (default 1e-12) */
    int32_t max_steps;  /* accepted + rejected steps per cell (default 100000) */
    int32_t mode;       /* SC_MODE_PLAIN, SC_MODE_PERSISTENT or SC_MODE_STATIC */
    int32_t tile;       /* persistent mode: cells per queue pull (default 1) */
    int32_t grid;       /* persistent/static modes: workgroups; 0 = resident capacity */
    int32_t order;      /* persistent mode: SC_ORDER_* (sorting needs a workspace
                           that sc_integrate allocates on first use) */
    int32_t fixed_step; /* 0: error-controlled steps (default); 1: steps of exactly
                           h_io[c] (h0[c] for sc_adjoint), the last one shortened to
                           end at dt, all accepted, no error control (h_io required) */
    double hmax_frac;   /* > 0: no step longer than hmax_frac * dt[c] (default 0: no
                           cap).  Error control sees only the state; a cap makes the
                           steps also resolve how perturbations relax, which the
                           adjoint's gradients then follow (see sc_adjoint) */
    int32_t reactor;    /* SC_REACTOR_CONST_P (default) or SC_REACTOR_CONST_V */
    int32_t method;     /* SC_METHOD_ROS4 (default) or SC_METHOD_EXTRAP */
    int32_t linalg;     /* SC_LINALG_AUTO (default), SC_LINALG_DENSE or SC_LINALG_SPARSE */
    int32_t cells_per_wave; /* sparse linear algebra: cells integrated side by side in
                           one 64-lane wave, 1, 2 or 4 (each cell then takes 64, 32 or 16
                           lanes, so N + 2 must fit them); 0 (default) = the most that
                           fit.  Other values, or more than 1 with the dense linear
                           algebra: SC_EINVAL.  Results agree with one cell per wave to
                           rounding (a cell's reductions and rate sums run over fewer
                           lanes in another order), not bit for bit. */
    /* Interpolated thermodynamics (paper Sec. 2.5: the chemistry library
     * interpolates costly thermodynamic functions with polynomials of
     * optimal degree; sparse linear algebra only).  thermo_tol > 0: each
     * reaction's -dG/RT and dH/RT are read from piecewise polynomials in
     * ln T over [thermo_Tmin, thermo_Tmax] (defaults 250 and 4000 K) with
     * at most thermo_tol absolute error (see sc_mech_thermo_fit) instead
     * of being summed from the species' NASA-7 values; a cell whose T is
     * outside the range uses the exact sums.  thermo_degree: the
     * polynomial degree, 0 (default) = the lowest whose table fits 4 MiB.
     * 0 (default) = exact.  The VJP and the adjoint refuse such a plan
     * (their derivatives follow the exact functions). */
    double thermo_tol;
    double thermo_Tmin, thermo_Tmax;
    int32_t thermo_degree;
} sc_options;

typedef struct {
    int32_t n_species, n_reactions, n_third_body, n_troe, n_elements;
    int32_t n_state;    /* N + 1 */
    int32_t n_padded;   /* register rows per cell used by the kernels */
    int32_t nnz_jac;    /* structural nonzeros of the (N+1)^2 Jacobian */
    int32_t nnz_lu;     /* nonzeros of L+U in the kernels' factorisation order */
    int32_t n_stages;   /* Rosenbrock stages per step */
    int32_t rhs_evals_per_step;
    int32_t exp_per_rhs;  /* exp/log/pow calls per right-hand side */
    int64_t flops_rhs;    /* per right-hand side, transcendental calls excluded */
    int64_t flops_jac;    /* analytical Jacobian assembly */
    int64_t flops_lu;     /* one factorisation as the kernel schedules it */
    int64_t flops_solve;  /* one forward + back substitution */
    int64_t flops_step;   /* one Rosenbrock step (Jacobian, LU, stages, control) */
    /* the sparse linear algebra (SC_LINALG_SPARSE), counted from its static
     * schedule: the bordered system of order N + 2 in minimum-degree order */
    int32_t nnz_a_sparse;       /* structural entries of the bordered matrix */
    int32_t nnz_lu_sparse;      /* entries of L + U (with fill) */
    int32_t lu_levels;          /* levels of the factorisation schedule */
    int32_t solve_levels;       /* levels of one forward + one backward solve */
    int64_t lu_updates_sparse;  /* Schur-complement updates of one factorisation */
    int64_t flops_lu_sparse;    /* one factorisation (division 1, fma 2) */
    int64_t flops_solve_sparse; /* one solve */
    int64_t flops_step_sparse;  /* one step with the sparse linear algebra */
    int32_t lu_tail_sparse;     /* trailing positions whose L+U block is full: factorised in
                                 * registers after the level schedule (its pivots are not in
                                 * lu_levels; flops_lu_sparse counts them) */
} sc_mech_info;

void sc_default_options(sc_options *opt);

/* Parse, validate and compile a mechanism (text format: see the package
 * docs; units of the rate law as in the paper's CHEMKIN-style mechanisms:
 * log10 A in cgs, Ea in J/mol).  Host only.  On error *out is NULL and
 * SC_EPARSE / SC_EUNSUPPORTED is returned with a message. */
sc_status sc_mech_load(const char *text, size_t len, sc_mech **out);
sc_status sc_mech_info_get(const sc_mech *mech, sc_mech_info *out);
/* index of a species by name, or SC_EINVAL */
sc_status sc_species_index(const sc_mech *mech, const char *name, int32_t *idx);

/* One array of the mechanism compiler's sparse algebra (paper Sec. 2.5:
 * sparse analytical Jacobian, sparse algebra management of the mechanism),
 * host memory, for inspection and tests.  With out == NULL only *bytes is
 * set (the size); else up to *bytes bytes are copied and *bytes is set to
 * the size.  Names (element type):
 *   "perm" (int32: position -> variable; species 0..N-1, N = T, N+1 = the
 *     border unknown sigma), "pattern" (uint8, N*N species-term pattern),
 *   "apat" (uint8, (N+2)^2 bordered pattern in positions),
 *   "erow", "ecol" (int32: row and column position of each L+U entry;
 *     entries are numbered column by column, rows ascending),
 *   "cstart" (int32, n + 1: first entry of each column), "cmask" (uint64,
 *     2 per column: bit i of word i / 64 set when row i has an entry),
 *   "sweep_f", "sweep_b" (uint32, n <= 64 only, 4 per column: mask of the
 *     rows below (above) the diagonal holding an entry, low and high word,
 *     and the first of those entries, then 0),
 *   "sweep_fi", "sweep_bi" (uint16, n <= 64 only, 64 per column k: the
 *     entry of row i in column k below (above) the diagonal, else nnz),
 *   "lu_b_lvl", "lu_c_lvl", "fw_lvl", "bw_lvl", "tfw_lvl", "tbw_lvl" (int32
 *     level offsets), "lu_b", "lu_u", "diag" (uint32 items), "lu_c", "fw",
 *     "bw", "tfw", "tbw" (uint64 items), "rxi" (uint16, RXI entries per
 *     reaction in mechanism order).
 * Item encodings: lu_b e_ik | e_kk << 16 (l_ik = a_ik / a_kk); lu_c
 * e_ij | e_ik << 16 | e_kj << 32 (a_ij -= l_ik u_kj); lu_u e_kj | k << 16
 * (u_kj /= u_kk); solves i | p << 16 | e << 32 (x_i -= a_e x_p).  lu_b and
 * lu_c hold the pivots before the dense tail only (sc_mech_info's
 * lu_tail_sparse): the last lu_tail_sparse pivots are eliminated densely
 * after the levels, with the same operations.
 * SC_EINVAL for an unknown name. */
sc_status sc_mech_sparse_array(const sc_mech *mech, const char *name, void *out, size_t *bytes);

/* The interpolation tables a plan with thermo_tol > 0 builds (host only).
 * For each reaction j (mechanism order) the functions
 *   F1_j(T) = -sum_k nu_kj g_k/(R T),  F2_j(T) = sum_k nu_kj h_k/(R T)
 * (nu: net coefficients; g, h from the NASA-7 data) are fitted in
 * u = ln T on nint equal intervals of [ln Tmin, ln Tmax]; on interval i the
 * polynomial of the degree in t = 2 (u - u_i) / du - 1 interpolates at the
 * Chebyshev points.  Each degree uses the fewest intervals whose largest
 * error on a check grid (3 (d+1) + 2 points per interval) is at most tol;
 * degree = 0 picks the lowest degree (1..8: the cheapest evaluation) whose
 * table fits 4 MiB (one die's L2 cache), a given degree may use up to 4096
 * intervals.  Out: *degree_out, *nint_out,
 * *max_err_out (that check-grid error); coef (may be NULL): nint * R * 2 *
 * (degree + 1) doubles [interval][reaction][function][power of t], up to
 * *ncoef of them, *ncoef set to the count.  SC_EINVAL for a bad range, tol or
 * degree, or when no degree reaches tol. */
sc_status sc_mech_thermo_fit(const sc_mech *mech, double Tmin, double Tmax, double tol, int32_t degree,
                             int32_t *degree_out, int32_t *nint_out, double *max_err_out, double *coef,
                             size_t *ncoef);
void sc_mech_free(sc_mech *mech);

/* Upload a mechanism's tables to a device (hipSetDevice(device) is made
 * current for the call) and pick the kernel variant. */
sc_status sc_plan_create(const sc_mech *mech, int device, const sc_options *opt, sc_plan **out);
void sc_plan_free(sc_plan *plan);

/* Right-hand side at n states (thermo, rates, production rates; the reactor
 * ODE of every cell): fT[c] = dT/dt, fY[k*ld + c] = dY_k/dt.  dlnA: R
 * per-reaction log multipliers of the net rate, or NULL. */
sc_status sc_rhs(sc_plan *plan, int64_t n, const double *T, const double *p, const double *Y,
                 int64_t ld, const double *dlnA, double *fT, double *fY, void *hip_stream);

/* Analytical Jacobian of the same right-hand side with respect to the state
 * (Y_0..Y_{N-1}, T): J[c*(N+1)*(N+1) + i*(N+1) + j] = d f_i / d y_j, with
 * index N standing for T. */
sc_status sc_jacobian(sc_plan *plan, int64_t n, const double *T, const double *p, const double *Y,
                      int64_t ld, const double *dlnA, double *J, void *hip_stream);

/* Solve (I/hg - J(y)) x = b per cell with the kernels' factorisation, where
 * hg[c] = h*gamma of the cell; b, x: [c*(N+1) + i] (state order as above). */
sc_status sc_linsolve(sc_plan *plan, int64_t n, const double *T, const double *p, const double *Y,
                      int64_t ld, const double *dlnA, const double *hg, const double *b, double *x,
                      void *hip_stream);

/* Integrate n cells over their own dt[c] (reactor model and method from the
 * plan's options: p[c] is the pressure, or the density of a constant-volume
 * reactor).  With SC_ORDER_COST, n_acc and n_rej are read (as the predicted
 * cost of each cell) before they are overwritten; they must then be non-NULL.
 *   in : T0[n], p[n], Y0[N*ld], dt[n], dlnA[R] or NULL,
 *        h_io[n] or NULL (initial step; the last accepted step is written back)
 *   out: T1[n], Y1[N*ld] (may alias T0/Y0), cell_status[n],
 *        n_acc[n], n_rej[n] (NULL allowed)
 * Options come from the plan (rtol, atol, max_steps, mode, tile, grid, order,
 * fixed_step, hmax_frac, reactor, method). */
sc_status sc_integrate(sc_plan *plan, int64_t n, const double *T0, const double *p, const double *Y0,
                       int64_t ld, const double *dt, const double *dlnA, double *h_io, double *T1,
                       double *Y1, int32_t *cell_status, int32_t *n_acc, int32_t *n_rej,
                       void *hip_stream);

/* sc_integrate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, options and results (bit for bit: the same kernels), but
 * the persistent mode's queue counter and cell-ordering workspace live in a
 * fixed device scratch array of the library (16 MiB per device, resolved on
 * the first call on each device and held until the process ends) instead of
 * plan allocations, so no call allocates or frees.  Limit: n <= 262,144
 * cells (SC_EINVAL beyond).  Every call on one device shares that scratch,
 * which keeps the last call's contents (the queue counter is cleared by a
 * kernel at the start of each call): calls that overlap on one device, on
 * different streams or host threads, race and must be serialised by the
 * caller.  Plain and static modes use no scratch. */
sc_status sc_integrate_noalloc(sc_plan *plan, int64_t n, const double *T0, const double *p, const double *Y0,
                               int64_t ld, const double *dt, const double *dlnA, double *h_io, double *T1,
                               double *Y1, int32_t *cell_status, int32_t *n_acc, int32_t *n_rej,
                               void *hip_stream);

/* Zonal reference-cell mapping (paper Sec. 2.5: the load-balanced solver the
 * paper builds on maps the chemistry solution of low-reactivity regions from
 * a reference cell instead of integrating every cell).  Low reactivity is a
 * mixture fraction below z_tol: Z = (beta - beta_ox) / (beta_fuel - beta_ox)
 * with Bilger's coupling function beta = sum_k (2 n_C,k + n_H,k / 2 -
 * n_O,k) Y_k / W_k (element atoms per species k; other elements do not
 * count), evaluated for the cell and for the two streams.  Zones are bands
 * of temperature of width dT (floor(T / dT) < ceil(SC_MAP_T_MAX / dT)) and,
 * when dlnp > 0, bands of ln(p / 1 Pa) of width dlnp (0 <= floor(ln p /
 * dlnp) < ceil(ln SC_MAP_P_MAX / dlnp)). */
#define SC_MAP_T_MAX 10000.0
#define SC_MAP_P_MAX 1e9
typedef struct {
    double z_tol; /* cells with Z < z_tol are mapped (finite) */
    double dT;    /* temperature band width [K], > 0 */
    double dlnp;  /* ln p band width, >= 0 (0: one band for every pressure) */
} sc_mapping;

/* Set the plan's mapping: the fuel and oxidiser stream compositions
 * (HOST arrays of N mass fractions) and the options above.  Allocates the
 * plan's zone table (64 MiB) on the first call.  SC_EINVAL for non-finite
 * or out-of-range options, streams with equal beta, or more than 2^24
 * zones. */
sc_status sc_plan_set_mapping(sc_plan *plan, const double *Y_fuel, const double *Y_ox, const sc_mapping *opt);

/* sc_integrate with the plan's mapping (set by sc_plan_set_mapping): a
 * mappable cell whose zone holds a mappable cell of lower index is not
 * integrated; the zone's lowest-index cell (its reference) is, and each
 * other cell of the zone takes the reference's change over the step scaled
 * by the ratio of the steps, as a mean rate:
 *   T1 = T0 + (T1_ref - T0_ref) dt / dt_ref, Y1 likewise per species,
 * with the reference's status and zero step counts (h_io is left as it
 * was).  Mapped cells need finite inputs and T, p, dt > 0.
 *   out: ref[n] (device): the reference of every cell (c itself when the
 *        cell was integrated), plus the sc_integrate outputs.
 * T1 and Y1 must not alias T0 and Y0 (SC_EINVAL).  The classification is a
 * few passes over the batch before the integration and one after it, on the
 * same stream; the launch options of the plan apply to the integrated
 * cells (the skipped ones cost a queue pull each). */
sc_status sc_integrate_mapped(sc_plan *plan, int64_t n, const double *T0, const double *p, const double *Y0,
                              int64_t ld, const double *dt, const double *dlnA, double *h_io, double *T1,
                              double *Y1, int32_t *cell_status, int32_t *n_acc, int32_t *n_rej, int32_t *ref,
                              void *hip_stream);

/* Vector-Jacobian product of the right-hand side (the transpose of the
 * sc_jacobian matrix applied to a weight): for every cell
 *   g = J(y)^T w,  with w = (wY[k*ld + c] for k < N, wT[c]) and the output
 *   in the same layout (gY, gT);
 * and, when g_dlnA_cell is not NULL, the parameter part
 *   g_dlnA_cell[j*n + c] = sum_i w_i d f_i / d dlnA_j
 * (dlnA_j multiplies the whole net rate of reaction j, forward and reverse
 * together, so this is q_j times the weight of reaction j's production
 * terms).  The building block of sc_adjoint (paper Sec. 2.5: analytical
 * Jacobian of the chemical source term), exposed for testing. */
sc_status sc_vjp(sc_plan *plan, int64_t n, const double *T, const double *p, const double *Y, int64_t ld,
                 const double *dlnA, const double *wT, const double *wY, double *gT, double *gY,
                 double *g_dlnA_cell, void *hip_stream);

/* Discrete adjoint of sc_integrate: the vector-Jacobian product of the map
 * (T0, Y0, dlnA) -> (T1, Y1) that the integrator computes, with its
 * accepted step sequence held fixed (the step-size controller is not
 * differentiated).  Gradients of the integrated source terms with respect to
 * the initial state and the rate constants (paper Sec. 2.1, Eqs. 3-4: the
 * sources come from the per-cell integration).
 *   in : the sc_integrate inputs (T0, p, Y0, ld, dt, dlnA; h0 = initial step
 *        per cell or NULL, read only) and the cotangents gT1[n], gY1[N*ld];
 *        cost[n] or NULL: predicted work per cell (e.g. the forward call's
 *        n_acc + n_rej), cells are then scheduled longest first;
 *        budget_bytes: device workspace cap (0 = 8 GiB).
 *   out: gT0[n], gY0[N*ld] (may alias gT1/gY1); g_dlnA[R] (sum over cells)
 *        or NULL; g_dlnA_cell[R*n] (layout [j*n + c]) or NULL; T1, Y1 (the
 *        recording pass's end state, identical to sc_integrate's) or NULL;
 *        cell_status[n]; n_acc[n] or NULL; *peak_bytes (workspace used) or
 *        NULL.
 * Each cell is integrated forward once more (recording step sizes and
 * checkpoints), then reversed step by step: every step is replayed from the
 * nearest stored state (a segment is recomputed from its checkpoint when not
 * every state fits), the stage equations are transposed (solves with the
 * step's own factors, J^T products at the stage points) and the derivative
 * of the iteration matrix contributes the second-order terms (exact
 * directional derivatives of J^T w).  The gradients are those of the
 * discrete map: where the controller takes steps much longer than the
 * relaxation times of a perturbed direction (a cell at equilibrium takes
 * one step), they differ from the continuous sensitivities by the method's
 * damping error for that direction; hmax_frac bounds the step and with it
 * that difference.  A cell whose integration fails gets its status and NaN
 * gradients (so g_dlnA is NaN).
 * The library sizes its per-wave workspace from max_steps; fewer waves run
 * when the budget is small; SC_EBUDGET if one wave does not fit.  The sum
 * over cells is taken in a fixed order: results do not depend on the
 * schedule. */
sc_status sc_adjoint(sc_plan *plan, int64_t n, const double *T0, const double *p, const double *Y0, int64_t ld,
                     const double *dt, const double *dlnA, const double *h0, const double *gT1, const double *gY1,
                     double *gT0, double *gY0, double *g_dlnA, double *g_dlnA_cell, const int32_t *cost,
                     double *T1, double *Y1, int32_t *cell_status, int32_t *n_acc, size_t budget_bytes,
                     size_t *peak_bytes, void *hip_stream);

/* Bytes of adjoint workspace per resident wave for the plan's max_steps. */
size_t sc_adjoint_slot_bytes(const sc_plan *plan);

/* Transport step of an operator-split driver on a uniform 2-D grid of
 * nx * ny cells (row-major, c = iy*nx + ix), every cell with its own local
 * time step dt[c] (paper Sec. 2.5: per-cell chemistry between flow steps,
 * local time stepping).  Not part of the chemistry integration: the cheap
 * mixing operator that alternates with sc_integrate in a split loop.
 * For each of ncomp components (rows of ld values, in[k*ld + c]):
 *   out = q - Co (q - q_west) + Fo (q_east + q_west + q_north + q_south - 4 q),
 *   Co = u[c] dt[c] / dx (first-order upwind, u >= 0 along +x),
 *   Fo = diffusivity dt[c] / dx^2,
 * with the inflow profile inflow[k*ny + iy] west of ix = 0 and zero-gradient
 * boundaries elsewhere.  With Co + 4 Fo <= 1 (the caller's choice of dt)
 * every output is a convex combination of inputs: mass fractions stay in
 * [0, 1] and keep their sum.  out has the layout of in (rows of ld values).
 * Device pointers; out must not alias in.  SC_EINVAL for non-positive
 * sizes, nx*ny*ncomp above 256 (2^31 - 1) (one thread per value in a grid of
 * 256-thread blocks), ld < nx*ny, NULL arrays, in == out,
 * dx <= 0 or diffusivity < 0. */
sc_status sc_transport2d(int32_t nx, int32_t ny, int32_t ncomp, const double *in, int64_t ld, const double *u,
                         const double *dt, double dx, double diffusivity, const double *inflow, double *out,
                         void *hip_stream);

/* Last error message of the calling thread (valid until its next call). */
const char *sc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
