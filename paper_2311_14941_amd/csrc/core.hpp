// Device building blocks shared by the forward and adjoint kernels: the
// Rosenbrock tableau, wave helpers, the per-cell LDS layout, thermodynamics,
// reaction rates with their analytical derivatives, the right-hand side and
// Jacobian passes, the in-register LU and the solves, one Rosenbrock attempt
// and the step-size controller.
//
// Work decomposition: one 64-lane wavefront integrates one cell (one
// independent homogeneous reactor, paper Sec. 1).  Inside the wave
//   - state, stage and error vectors are lane-distributed: lane i holds
//     component i of (Y_0..Y_{N-1}, T), so vector algebra is one VALU op;
//   - thermodynamics runs with lanes over species, rates and their analytical
//     derivatives with lanes over reactions (Sec. 2.5: sparse analytical
//     Jacobian), scattering into LDS with LDS floating-point atomics;
//   - the iteration matrix I/(h gamma) - J is formed in VGPRs, row i in lane
//     i, factorised without pivoting in a fixed order by a fully unrolled
//     right-looking LU whose pivot rows are broadcast with readlane, and then
//     parked in LDS (column-major, conflict-free) for the triangular solves;
//   - the Rosenbrock stepper and its error/step-size controller run uniformly
//     per wave (no divergence: every lane follows its cell's control flow).
// Everything is FP64.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "devmech.hpp"

namespace scdev {


// ---------------------------------------------------------------------------
// Rosenbrock tableau (transformed form; derivation in tableau.py, ros4()):
// 4 stages, order 4, L-stable, embedded order 3; stage 4 is evaluated at the
// stage-3 point, so a step costs 3 function evaluations (one of them in the
// Jacobian pass), 1 factorisation and 4 solves.
// ---------------------------------------------------------------------------
constexpr int NS = 4;
constexpr double GAM = 0.572816062482135;
static __constant__ double TA[NS][NS] = {{0.0, 0.0, 0.0, 0.0},
                                  {1.0474566606950075, 0.0, 0.0, 0.0},
                                  {1.5266834054578882, 0.49110997987229194, 0.0, 0.0},
                                  {1.5266834054578882, 0.49110997987229194, 0.0, 0.0}};
static __constant__ double TC[NS][NS] = {{0.0, 0.0, 0.0, 0.0},
                                  {-2.8287104387961546, 0.0, 0.0, 0.0},
                                  {-1.1423273772481277, 0.9544101947030211, 0.0, 0.0},
                                  {-3.972521690537523, -0.6901523982223108, -1.548869644699513, 0.0}};
static __constant__ double TM[NS] = {2.326763557172835, -0.7953731300411474, 1.6632540048577067, 1.0474566606950075};
static __constant__ double TE[NS] = {0.4092508278871161, -1.0795845833425672, 0.9649495643943683,
                              1.0474566606950078};  // m - mhat
// function value of a stage: 0 = f(y) from the Jacobian pass, -1 = evaluate,
// k > 0 = reuse the value evaluated at stage k (same point)
static __constant__ int TREUSE[NS] = {0, -1, -1, 2};
// step-size exponent 1/(embedded order + 1) = 1/4 (ctl_end takes the fourth root)

constexpr int WAVE = 64;
// LDS loads issued ahead per group in the unrolled row/solve loops; bounds
// the scheduler's hoisting (register pressure) while keeping latency hidden
constexpr int LD_GROUP = 8;
#define SC_FENCE_EVERY(i) \
    if (((i) + 1) % LD_GROUP == 0) __builtin_amdgcn_sched_barrier(0)

// ---------------------------------------------------------------------------
// wave helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rdlane(double v, int lane)
{
    int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

__device__ __forceinline__ void wave_sync() { __syncthreads(); }

// ---------------------------------------------------------------------------
// Dual numbers (value, directional derivative): the chemistry below is
// written once for a scalar type S; S = double is the integrator, S = Dual
// carries an exact directional derivative through the same arithmetic (used
// by the adjoint for the derivative of the Jacobian along a direction).
// ---------------------------------------------------------------------------
// (the double overloads stay visible next to the Dual ones below)
using ::exp;
using ::log;
using ::log10;

struct Dual {
    double v, d;
    Dual() = default;
    __host__ __device__ constexpr Dual(double x) : v(x), d(0.0) {}
    __host__ __device__ constexpr Dual(double x, double t) : v(x), d(t) {}
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator-(Dual a) { return {-a.v, -a.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, fma(a.d, b.v, a.v * b.d)}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b)
{
    const double q = a.v / b.v;
    return {q, (a.d - q * b.d) / b.v};
}
__device__ __forceinline__ Dual operator+(Dual a, double b) { return {a.v + b, a.d}; }
__device__ __forceinline__ Dual operator+(double a, Dual b) { return {a + b.v, b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, double b) { return {a.v - b, a.d}; }
__device__ __forceinline__ Dual operator-(double a, Dual b) { return {a - b.v, -b.d}; }
__device__ __forceinline__ Dual operator*(Dual a, double b) { return {a.v * b, a.d * b}; }
__device__ __forceinline__ Dual operator*(double a, Dual b) { return {a * b.v, a * b.d}; }
__device__ __forceinline__ Dual operator/(Dual a, double b) { return {a.v / b, a.d / b}; }
__device__ __forceinline__ Dual operator/(double a, Dual b)
{
    const double q = a / b.v;
    return {q, -q * b.d / b.v};
}
__device__ __forceinline__ Dual &operator+=(Dual &a, Dual b) { return a = a + b; }
__device__ __forceinline__ Dual &operator-=(Dual &a, Dual b) { return a = a - b; }
__device__ __forceinline__ Dual &operator*=(Dual &a, Dual b) { return a = a * b; }
__device__ __forceinline__ Dual exp(Dual a)
{
    const double e = exp(a.v);
    return {e, e * a.d};
}
__device__ __forceinline__ Dual log(Dual a) { return {log(a.v), a.d / a.v}; }
__device__ __forceinline__ Dual log10(Dual a) { return {log10(a.v), a.d / (a.v * 2.302585092994046)}; }
__device__ __forceinline__ Dual rdlane(Dual v, int lane) { return {rdlane(v.v, lane), rdlane(v.d, lane)}; }
__device__ __forceinline__ Dual wave_sum(Dual v) { return {wave_sum(v.v), wave_sum(v.d)}; }

// the part a pass reports: the value (S = double) or the derivative (Dual)
__device__ __forceinline__ double part(double x) { return x; }
__device__ __forceinline__ double part(Dual x) { return x.d; }
__device__ __forceinline__ double value(double x) { return x; }
__device__ __forceinline__ double value(Dual x) { return x.v; }

// LDS access of a scalar: a Dual's derivative lives toff doubles from its value
template <class S>
__device__ __forceinline__ S lds_get(const double *lds, int i, int toff);
template <>
__device__ __forceinline__ double lds_get<double>(const double *lds, int i, int)
{
    return lds[i];
}
template <>
__device__ __forceinline__ Dual lds_get<Dual>(const double *lds, int i, int toff)
{
    return {lds[i], lds[i + toff]};
}
__device__ __forceinline__ void lds_put(double *lds, int i, double x, int) { lds[i] = x; }
__device__ __forceinline__ void lds_put(double *lds, int i, Dual x, int toff)
{
    lds[i] = x.v;
    lds[i + toff] = x.d;
}
__device__ __forceinline__ void lds_add(double *lds, int i, double x, int) { atomicAdd(&lds[i], x); }
__device__ __forceinline__ void lds_add(double *lds, int i, Dual x, int toff)
{
    atomicAdd(&lds[i], x.v);
    atomicAdd(&lds[i + toff], x.d);
}

// The reactor model as a compile-time constant.  Every device routine is
// inlined into its kernel, so a kernel that calls this on its DevMech
// argument gets the branches on m.cv folded away.
template <bool CV>
__device__ __forceinline__ DevMech fix_reactor(DevMech m)
{
    m.cv = CV ? 1 : 0;
    return m;
}

// ---------------------------------------------------------------------------
// LDS layout of one cell (doubles)
// ---------------------------------------------------------------------------
template <int NP>
struct Lds {
    // row stride of the Jacobian terms: lanes reading their own rows hit
    // addresses a stride apart; an odd stride spreads them over the banks
    static constexpr int PS = NP + 1;
    static constexpr int P = 0;          // NP x PS Jacobian terms, later the LU factors (stride NP)
    // the term region is also where the adjoint's dual passes keep the
    // derivatives of C, G, H, WD and of its own V vector (each at a fixed
    // offset -C from the value), which ends 8 NP + NS WAVE doubles in
    static constexpr int PREG = NP * PS > 8 * NP + NS * WAVE ? NP * PS : 8 * NP + NS * WAVE;
    static constexpr int C = PREG;       // concentrations
    static constexpr int G = C + NP;     // g/RT
    static constexpr int H = G + NP;     // h/RT
    static constexpr int WD = H + NP;    // production-rate accumulator
    static constexpr int UA = WD + NP;   // Euler-term accumulator
    static constexpr int IW = UA + NP;   // 1/W_c (0 for c >= N)
    static constexpr int U = IW + NP;    // NS stage vectors, WAVE apart
    static constexpr int SIZE = U + NS * WAVE;
};

// Per-cell uniform quantities at the point where a right-hand side was taken.
// p is the pressure; cp the heat capacity of the reactor's energy balance
// (c_p at constant pressure, c_v at constant volume).
template <class S = double>
struct Mix {
    S T, invT, lnT;
    double p;
    S rho, Wbar, cp;
};

template <class S = double>
struct Thermo {
    S cpR, hRT, sR, dcpR;
};

// NASA-7 of species k (single temperature range)
template <class S>
__device__ __forceinline__ Thermo<S> nasa7(const DevMech &m, int k, S T, S lnT, S invT)
{
    const int N = m.N;
    const double *a = m.nasa();
    const double a0 = a[k], a1 = a[N + k], a2 = a[2 * N + k], a3 = a[3 * N + k], a4 = a[4 * N + k],
                 a5 = a[5 * N + k], a6 = a[6 * N + k];
    Thermo<S> t;
    t.cpR = a0 + T * (a1 + T * (a2 + T * (a3 + T * a4)));
    t.hRT = a0 + T * (a1 * 0.5 + T * (a2 * (1.0 / 3.0) + T * (a3 * 0.25 + T * a4 * 0.2))) + a5 * invT;
    t.sR = a0 * lnT + T * (a1 + T * (a2 * 0.5 + T * (a3 * (1.0 / 3.0) + T * a4 * 0.25))) + a6;
    t.dcpR = a1 + T * (2.0 * a2 + T * (3.0 * a3 + T * 4.0 * a4));
    return t;
}

// Mixture state from the lane-distributed y (lane k < N: Y_k, lane N: T);
// writes C, g/RT, h/RT to LDS and clears the accumulators.  With S = Dual
// the derivatives go toff doubles beyond the values.  p is the pressure, or
// in a constant-volume reactor the density.
template <int NP, class S = double>
__device__ __forceinline__ Mix<S> mixture(const DevMech &m, double *lds, S y, double p, Thermo<S> &th, int lane,
                                          int toff = 0)
{
    const int N = m.N;
    Mix<S> x;
    x.T = rdlane(y, N);
    x.invT = 1.0 / x.T;
    x.lnT = log(x.T);
    x.p = p;
    S yw = 0.0, cpw = 0.0;
    th = Thermo<S>{0.0, 0.0, 0.0, 0.0};
    if (lane < N) {
        th = nasa7<S>(m, lane, x.T, x.lnT, x.invT);
        yw = y * m.invW()[lane];
        cpw = th.cpR * yw;
    }
    x.Wbar = 1.0 / wave_sum(yw);
    x.cp = m.Rgas * wave_sum(cpw);
    if (m.cv) {
        x.rho = p;
        x.p = value(p * m.Rgas * x.T / x.Wbar);
        x.cp = x.cp - m.Rgas / x.Wbar;
    } else {
        x.rho = p * x.Wbar * x.invT / m.Rgas;
    }
    if (lane < N) {
        lds_put(lds, Lds<NP>::C + lane, x.rho * yw, toff);
        lds_put(lds, Lds<NP>::G + lane, th.hRT - th.sR, toff);
        lds_put(lds, Lds<NP>::H + lane, th.hRT, toff);
        lds_put(lds, Lds<NP>::WD + lane, S(0.0), toff);
        lds[Lds<NP>::UA + lane] = 0.0;
    }
    if (m.cv && lane == N) lds[Lds<NP>::UA + N] = 0.0;  // temperature-row accumulator (constant volume)
    return x;
}

template <class S>
__device__ __forceinline__ S ipow(S c, int nu)
{
    S r = c;
    if (nu >= 2) r *= c;
    if (nu >= 3) r *= c;
    return r;
}
template <class S>
__device__ __forceinline__ S dipow(S c, int nu)  // d(c^nu)/dc
{
    return nu == 1 ? S(1.0) : nu == 2 ? 2.0 * c : 3.0 * c * c;
}

// One reaction's rate of progress and, in the Jacobian pass, its derivatives
// with respect to the slot species' concentrations and to T.  Slots: 0..2
// reactants, 3..5 products, 6..9 enhanced third-body species.
template <class S = double>
struct RxOut {
    S q;             // net rate of progress (mol/m^3/s)
    S d[sc::NDEP];   // dq/dC of slot species
    S dT;            // dq/dT at fixed C
    S euler;         // q - sum_s C_s dq/dC_s
    S dH;            // reaction enthalpy / RT
};

// A reaction's record in registers: one burst of wide loads issued together
// (one memory round trip), so later uses of its fields wait on nothing.
__device__ __forceinline__ RxRec load_rec(const DevMech &m, int j)
{
    RxRec r;
    __builtin_memcpy(&r, &m.rx[j], sizeof(RxRec));
    return r;
}

// Horner evaluation of the degree-d polynomial with coefficients c[0..d] at t
__device__ __forceinline__ double poly_t(const double *c, int d, double t)
{
    double p = c[d];
#pragma unroll 1
    for (int q = d - 1; q >= 0; --q) p = fma(p, t, c[q]);
    return p;
}

// itc: with interpolated thermodynamics, this reaction's coefficients of
// -dG/RT and dH/RT (degree ideg each, in the local coordinate it of the
// cell's ln T interval) replace the sums over the species' g/RT and h/RT
template <bool JAC, class S = double>
__device__ __forceinline__ RxOut<S> reaction(const DevMech &m, const double *lds, const RxRec &rr, const Mix<S> &x,
                                             double dl, int CO, int GO, int HO, int toff = 0,
                                             const double *itc = nullptr, double it = 0.0, int ideg = 0)
{
    const int kind = rr.kind;
    const int nr = rr.nr, np = rr.np;
    const S lnkinf = rr.lnA + dl + rr.b * x.lnT - rr.EaR * x.invT;
    const S kinf = exp(lnkinf);
    int rn[sc::MAXSIDE], pn[sc::MAXSIDE];
    S rc[sc::MAXSIDE], pc[sc::MAXSIDE];
    S dG = 0.0, dH = 0.0;
#pragma unroll
    for (int i = 0; i < sc::MAXSIDE; ++i) {
        const bool ur = i < nr, up = i < np;
        const int rs = ur ? rr.rsp[i] : 0;
        const int ps = up ? rr.psp[i] : 0;
        rn[i] = ur ? rr.rnu[i] : 0;
        pn[i] = up ? rr.pnu[i] : 0;
        rc[i] = ur ? lds_get<S>(lds, CO + rs, toff) : S(1.0);
        pc[i] = up ? lds_get<S>(lds, CO + ps, toff) : S(1.0);
        if (itc) continue;
        dG += pn[i] * (up ? lds_get<S>(lds, GO + ps, toff) : S(0.0)) -
              rn[i] * (ur ? lds_get<S>(lds, GO + rs, toff) : S(0.0));
        if (JAC)
            dH += pn[i] * (up ? lds_get<S>(lds, HO + ps, toff) : S(0.0)) -
                  rn[i] * (ur ? lds_get<S>(lds, HO + rs, toff) : S(0.0));
    }
    if (itc) {
        dG = -poly_t(itc, ideg, it);
        if (JAC) dH = poly_t(itc + ideg + 1, ideg, it);
    }
    const int dnu = rr.dnu;
    const S lnKc = -dG + dnu * (m.lnp0R - x.lnT);
    // third-body concentration, rewritten with sum_k C_k = p/(R T):
    // [M] = p/(RT) + sum_enhanced (alpha - 1) C.  At constant pressure p/(RT)
    // depends on T alone; at constant volume it is rho/Wbar, a function of
    // every C_k (dM/dC_k = 1, the rank-one part the caller adds)
    S M = 0.0;
    const int ne = rr.neff;
    S ec[sc::MAXENH];
    double ea[sc::MAXENH];
#pragma unroll
    for (int e = 0; e < sc::MAXENH; ++e) {
        const bool ue = e < ne;
        ea[e] = ue ? rr.eam1[e] : 0.0;
        ec[e] = ue ? lds_get<S>(lds, CO + rr.esp[e], toff) : S(0.0);
    }
    if (kind != sc::RX_PLAIN) {
        M = x.p * x.invT / m.Rgas;
#pragma unroll
        for (int e = 0; e < sc::MAXENH; ++e) M += ea[e] * ec[e];
    }
    S kf = kinf, phi = 0.0, dlnF_T = 0.0, dlnk0 = 0.0;
    if (kind == sc::RX_TROE) {
        const TroeRec &tr = m.troe[rr.tix];
        const S lnk0 = tr.lnA0 + dl + tr.b0 * x.lnT - tr.Ea0R * x.invT;
        const S Pr = exp(lnk0 - lnkinf) * M;
        const double a = tr.a, iT3 = tr.iT3, iT1 = tr.iT1, T2 = tr.T2;
        const S e3 = exp(-x.T * iT3), e1 = exp(-x.T * iT1), e2 = exp(-T2 * x.invT);
        const S Fc = (1.0 - a) * e3 + a * e1 + e2;
        const S L = log10(Fc);
        const S cc = -0.4 - 0.67 * L, nn = 0.75 - 1.27 * L;
        const S X = log10(Pr) + cc;
        const S D = nn - 0.14 * X;
        const S f = X / D;
        const S opf = 1.0 + f * f;
        const S lF = L / opf;
        kf = kinf * (Pr / (1.0 + Pr)) * exp(2.302585092994046 * lF);
        if (JAC) {
            const S g = -L * 2.0 * f / (opf * opf);
            phi = 1.0 / (1.0 + Pr) + g * (nn / (D * D));  // dln kf / dln Pr
            const S dlF_dL = 1.0 / opf + g * ((-0.67 * nn + 1.27 * X) / (D * D));
            const S dFc = -(1.0 - a) * iT3 * e3 - a * iT1 * e1 + T2 * x.invT * x.invT * e2;
            dlnF_T = dlF_dL * dFc / Fc;  // dln F/dT at fixed Pr
            dlnk0 = (tr.b0 + tr.Ea0R * x.invT) * x.invT;
        }
    }
    const S kr = kf * exp(-lnKc);
    const S p0 = ipow(rc[0], rn[0]), p1 = ipow(rc[1], rn[1]), p2 = ipow(rc[2], rn[2]);
    const S s0 = ipow(pc[0], pn[0]), s1 = ipow(pc[1], pn[1]), s2 = ipow(pc[2], pn[2]);
    const S Rf = kf * (p0 * p1 * p2), Rr = kr * (s0 * s1 * s2);
    const S q0 = Rf - Rr;
    RxOut<S> o;
    o.q = kind == sc::RX_THIRD ? q0 * M : q0;
    if (!JAC) return o;
    const S fsc = kind == sc::RX_THIRD ? M : S(1.0);
    o.d[0] = nr > 0 ? fsc * kf * dipow(rc[0], rn[0]) * p1 * p2 : S(0.0);
    o.d[1] = nr > 1 ? fsc * kf * dipow(rc[1], rn[1]) * p0 * p2 : S(0.0);
    o.d[2] = nr > 2 ? fsc * kf * dipow(rc[2], rn[2]) * p0 * p1 : S(0.0);
    o.d[3] = np > 0 ? -fsc * kr * dipow(pc[0], pn[0]) * s1 * s2 : S(0.0);
    o.d[4] = np > 1 ? -fsc * kr * dipow(pc[1], pn[1]) * s0 * s2 : S(0.0);
    o.d[5] = np > 2 ? -fsc * kr * dipow(pc[2], pn[2]) * s0 * s1 : S(0.0);
    const S dlnkinf = (rr.b + rr.EaR * x.invT) * x.invT;
    const S dlnKc = (dH - dnu) * x.invT;
    const S dMdT = m.cv ? S(0.0) : -x.p * x.invT * x.invT / m.Rgas;
    S dqM = 0.0;  // dq/d[M]
    S dlnkf = dlnkinf;
    if (kind == sc::RX_THIRD) {
        dqM = q0;
    } else if (kind == sc::RX_TROE) {
        dqM = q0 * phi / M;
        dlnkf = dlnkinf + phi * (dlnk0 - dlnkinf + dMdT / M) + dlnF_T;
    }
    S dT = q0 * dlnkf + Rr * dlnKc;
    if (kind == sc::RX_THIRD) dT = M * dT + q0 * dMdT;
#pragma unroll
    for (int e = 0; e < sc::MAXENH; ++e) o.d[6 + e] = dqM * ea[e];
    o.dT = dT;
    S eu = o.q;
#pragma unroll
    for (int i = 0; i < sc::MAXSIDE; ++i)
        eu -= (i < nr ? rc[i] : S(0.0)) * o.d[i] + (i < np ? pc[i] : S(0.0)) * o.d[3 + i];
#pragma unroll
    for (int e = 0; e < sc::MAXENH; ++e) eu -= ec[e] * o.d[6 + e];
    // constant pressure: the Euler remainder; constant volume: dq/d[M], the
    // weight of the rank-one part of dq/dC
    o.euler = m.cv ? dqM : eu;
    o.dH = dH;
    return o;
}

// Scatter a reaction's contributions: production rates (always) and, in the
// Jacobian pass, the sparse analytical terms of every (row, slot) pair, the
// temperature column and (weighted by the reaction enthalpy) the temperature row.
template <int NP, bool JAC>
__device__ __forceinline__ void scatter(const DevMech &m, double *lds, const RxRec &rr, const RxOut<> &o, double dHJ)
{
    const int N = m.N;
    const int nr = rr.nr, np = rr.np;
    double *P = lds + Lds<NP>::P;
    int col[sc::NDEP];
    bool use[sc::NDEP];
    if (JAC) {
        const int ne = rr.neff;
#pragma unroll
        for (int i = 0; i < sc::MAXSIDE; ++i) {
            use[i] = i < nr;
            col[i] = use[i] ? rr.rsp[i] : 0;
            use[3 + i] = i < np;
            col[3 + i] = use[3 + i] ? rr.psp[i] : 0;
        }
#pragma unroll
        for (int e = 0; e < sc::MAXENH; ++e) {
            use[6 + e] = e < ne;
            col[6 + e] = use[6 + e] ? rr.esp[e] : 0;
        }
    }
    // rows: reactants then products, unrolled over the slots so that the
    // record's species and coefficients stay in registers (a rolled loop
    // indexes them at run time and reloads them from memory every row)
#pragma unroll
    for (int r = 0; r < 2 * sc::MAXSIDE; ++r) {
        const bool isr = r < sc::MAXSIDE;
        const int ri = isr ? r : r - sc::MAXSIDE;
        if (ri >= (isr ? nr : np)) continue;
        const int row = isr ? rr.rsp[ri] : rr.psp[ri];
        const double nu = isr ? -(double)rr.rnu[ri] : (double)rr.pnu[ri];
        atomicAdd(&lds[Lds<NP>::WD + row], nu * o.q);
        if (JAC) {
            atomicAdd(&lds[Lds<NP>::UA + row], nu * o.euler);
            double *Prow = P + row * Lds<NP>::PS;
#pragma unroll
            for (int s = 0; s < sc::NDEP; ++s)
                if (use[s]) atomicAdd(&Prow[col[s]], nu * o.d[s]);
            atomicAdd(&Prow[N], nu * o.dT);
        }
    }
    if (JAC) {
#pragma unroll
        for (int s = 0; s < sc::NDEP; ++s)
            if (use[s]) atomicAdd(&P[N * Lds<NP>::PS + col[s]], dHJ * o.d[s]);
        atomicAdd(&P[N * Lds<NP>::PS + N], dHJ * o.dT);
        if (m.cv) atomicAdd(&lds[Lds<NP>::UA + N], dHJ * o.euler);
    }
}

// Right-hand side f(y), lane-distributed (0 in padding lanes).
template <int NP>
__device__ double rhs(const DevMech &m, double *lds, double y, double p, const double *dlnA, int lane)
{
    const int N = m.N, R = m.R;
    Thermo<> th;
    const Mix<> x = mixture<NP>(m, lds, y, p, th, lane);
    wave_sync();
#pragma unroll 1
    for (int j = lane; j < R; j += WAVE) {
        const RxRec rr = load_rec(m, j);
        const double dl = dlnA ? dlnA[rr.orig] : 0.0;
        const RxOut<> o = reaction<false>(m, lds, rr, x, dl, Lds<NP>::C, Lds<NP>::G, Lds<NP>::H);
        scatter<NP, false>(m, lds, rr, o, 0.0);
    }
    wave_sync();
    double f = 0.0, hw = 0.0;
    if (lane < N) {
        const double wd = lds[Lds<NP>::WD + lane];
        f = m.W()[lane] * wd / x.rho;
        hw = (m.cv ? th.hRT - 1.0 : th.hRT) * wd;  // h_k/RT, or u_k/RT at constant volume
    }
    const double H = m.Rgas * x.T * wave_sum(hw);
    if (lane == N) f = -H / (x.rho * x.cp);
    wave_sync();
    return f;
}

// Per-lane coefficients turning row `lane` of the finalised LDS terms into a
// Jacobian row:  J[c] = IW[c] (alpha P[c] + beta) + [c == N] (alphaT P[c] + betaT).
struct RowCoef {
    double alpha, beta, alphaT, betaT;
};

// Jacobian pass: f(y) plus the analytical terms, finalised in LDS.
template <int NP>
__device__ double rhs_jac(const DevMech &m, double *lds, double y, double p, const double *dlnA, int lane,
                          RowCoef &rc)
{
    const int N = m.N, R = m.R;
    double *P = lds + Lds<NP>::P;
    Thermo<> th;
    const Mix<> x = mixture<NP>(m, lds, y, p, th, lane);
    if (lane < NP) {
#pragma unroll 4
        for (int i = 0; i < NP; ++i) P[i * Lds<NP>::PS + lane] = 0.0;  // lane c clears column c
    }
    wave_sync();
    const double RT = m.Rgas * x.T;
#pragma unroll 1
    for (int j = lane; j < R; j += WAVE) {
        const RxRec rr = load_rec(m, j);
        const double dl = dlnA ? dlnA[rr.orig] : 0.0;
        const RxOut<> o = reaction<true>(m, lds, rr, x, dl, Lds<NP>::C, Lds<NP>::G, Lds<NP>::H);
        // temperature-row weight: the reaction's enthalpy, or at constant
        // volume its internal energy (dH - dnu) R T
        scatter<NP, true>(m, lds, rr, o, m.cv ? (o.dH - rr.dnu) * RT : o.dH * RT);
    }
    wave_sync();
    // m.cv: the energy balance is on u_k = h_k - R T, the heat capacity c_v
    const double one = m.cv ? 1.0 : 0.0;
    double f = 0.0, hw = 0.0, eu = 0.0, cpf = 0.0, dcp = 0.0, uk = 0.0, ua = 0.0, Wk = 0.0;
    if (lane < N) {
        Wk = m.W()[lane];
        const double iw = m.invW()[lane];
        const double wd = lds[Lds<NP>::WD + lane];
        ua = lds[Lds<NP>::UA + lane];
        f = Wk * wd / x.rho;
        uk = Wk * ua / x.rho;
        hw = (th.hRT - one) * wd;
        eu = th.hRT * uk * iw;           // (h_k/(R T W_k)) u_k
        cpf = (th.cpR - one) * f * iw;   // cp_k/(R W_k) f_k (cv_k at constant volume)
        dcp = th.dcpR * y * iw;          // dcp_k/dT/(R W_k) Y_k
    }
    const double H = RT * wave_sum(hw);
    const double Eu = m.cv ? 0.0 : RT * wave_sum(eu);  // sum_k (h_k/W_k) u_k
    const double Scpf = m.Rgas * wave_sum(cpf);
    const double Sdcp = m.Rgas * wave_sum(dcp);
    const double fT = -H / (x.rho * x.cp);
    if (lane == N) f = fT;
    // fold the column-dependent parts of the temperature row into P[N][*].
    // Constant pressure:
    //   J_Tm = -(1/cp) (1/W_m) (P_Tm + Wbar Eu + fT cp_m),
    //   J_TT = -(1/cp) (P_TT/rho + Eu/T + sum cp_k f_k/W_k + fT sum dcp_k Y_k/W_k);
    // constant volume (C_k = rho Y_k/W_k, no density border; the rank-one
    // part of d[M]/dC accumulated in UA[N] for this row, UA[k] for row k):
    //   J_Tm = -(1/cv) (1/W_m) (P_Tm + UA_N + fT cv_m),
    //   J_TT = -(1/cv) (P_TT/rho + sum cv_k f_k/W_k + fT sum dcp_k Y_k/W_k)
    const int PS = Lds<NP>::PS;
    const double tb = m.cv ? lds[Lds<NP>::UA + N] : x.Wbar * Eu;
    if (lane < N) P[N * PS + lane] += tb + fT * m.Rgas * (th.cpR - one);
    if (lane == N) P[N * PS + N] = P[N * PS + N] / x.rho + Eu * x.invT + Scpf + fT * Sdcp;
    if (lane < NP) lds[Lds<NP>::IW + lane] = lane < N ? m.invW()[lane] : 0.0;
    wave_sync();
    const double invcp = 1.0 / x.cp;
    if (lane < N) {
        // species rows, constant pressure: J_km = (W_k/W_m) P_km + u_k Wbar/W_m,
        // J_kT = (W_k/rho) P_kT + u_k/T; constant volume: J_km = (W_k/W_m)
        // (P_km + UA_k), J_kT = (W_k/rho) P_kT
        rc = m.cv ? RowCoef{Wk, Wk * ua, Wk / x.rho, 0.0} : RowCoef{Wk, uk * x.Wbar, Wk / x.rho, uk * x.invT};
    } else if (lane == N) {
        rc = RowCoef{-invcp, 0.0, -invcp, 0.0};
    } else {
        rc = RowCoef{0.0, 0.0, 0.0, 0.0};
    }
    return f;
}

// Row `lane` of J from the finalised LDS terms into registers.
template <int NP>
__device__ __forceinline__ void jac_row(const DevMech &m, const double *lds, const RowCoef &rc, int lane,
                                        double (&a)[NP])
{
    const int N = m.N;
    const double *P = lds + Lds<NP>::P + (lane < NP ? lane : 0) * Lds<NP>::PS;
    const double *IW = lds + Lds<NP>::IW;
#pragma unroll
    for (int c = 0; c < NP; ++c) {
        const double pv = P[c];
        const double t = c == N ? fma(rc.alphaT, pv, rc.betaT) : 0.0;
        a[c] = fma(IW[c], fma(rc.alpha, pv, rc.beta), t);
        SC_FENCE_EVERY(c);
    }
}

// M = I/hg - J into registers (padding rows get the identity).
template <int NP>
__device__ __forceinline__ void form_matrix(const DevMech &m, const double *lds, const RowCoef &rc, int lane,
                                            double inv_hg, double (&a)[NP])
{
    jac_row<NP>(m, lds, rc, lane, a);
    const int n = m.N + 1;
    const double diag = lane < n ? inv_hg : 1.0;
#pragma unroll
    for (int c = 0; c < NP; ++c) a[c] = c == lane ? diag - a[c] : -a[c];
}

// In-register LU without pivoting, natural order; row i in lane i.  After the
// call a[k] (k < lane) holds L (unit diagonal implied), a[k] (k >= lane) U,
// and dinv = 1/U_ii.
template <int NP>
__device__ __forceinline__ void lu_factor(double (&a)[NP], double &dinv, int lane)
{
    dinv = 0.0;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const double piv = rdlane(a[k], k);
        const double inv = 1.0 / piv;
        if (lane == k) dinv = inv;
        const bool below = lane > k;
        const double l = below ? a[k] * inv : 0.0;
        if (below) a[k] = l;
#pragma unroll
        for (int j = k + 1; j < NP; ++j) {
            const double u = rdlane(a[j], k);
            a[j] = fma(-l, u, a[j]);
            SC_FENCE_EVERY(j - k - 1);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Park the factors in LDS, column-major (F[c*PS + i] = row i, column c), so
// that every read in the triangular solves is one contiguous wave access.
template <int NP>
__device__ __forceinline__ void store_factors(double *F, const double (&a)[NP], int lane)
{
    if (lane < NP) {
#pragma unroll
        for (int c = 0; c < NP; ++c) {
            F[c * Lds<NP>::PS + lane] = a[c];
            SC_FENCE_EVERY(c);
        }
    }
}

// Solve (L U) x = b with the factors in LDS; b lane-distributed.
template <int NP>
__device__ __forceinline__ double lu_solve(const double *F, double dinv, double b, int lane)
{
    const int li = lane < NP ? lane : 0;
#pragma unroll
    for (int k = 0; k < NP - 1; ++k) {
        const double l = F[k * Lds<NP>::PS + li];
        const double z = rdlane(b, k);
        if (lane > k) b = fma(-l, z, b);
        SC_FENCE_EVERY(k);
    }
#pragma unroll
    for (int k = NP - 1; k >= 0; --k) {
        if (lane == k) b *= dinv;
        const double z = rdlane(b, k);
        const double u = F[k * Lds<NP>::PS + li];
        if (lane < k) b = fma(-u, z, b);
        SC_FENCE_EVERY(NP - 1 - k);
    }
    return lane < NP ? b : 0.0;
}

// Form, factorise and park M = I/hg - J in F (the LDS term region itself,
// or per-cell global scratch); returns 1/U_ii of this lane.
template <int NP>
__device__ __forceinline__ double factor_matrix(const DevMech &m, double *lds, const RowCoef &rc, int lane,
                                                double inv_hg, double *F)
{
    double dinv;
    double a[NP];
    form_matrix<NP>(m, lds, rc, lane, inv_hg, a);
    lu_factor<NP>(a, dinv, lane);
    wave_sync();  // every lane has read its row of the terms
    store_factors<NP>(F, a, lane);
    wave_sync();
    return dinv;
}

// One Rosenbrock attempt of size hc from y: Jacobian pass, factorisation
// (parked in F), the four stages (stage vectors u_i left in LDS) and the
// embedded error.  Returns the new state; *err gets the scaled RMS error.
// Forward integration and adjoint replay both call this, so a replayed
// step reproduces the recorded one bit for bit.
template <int NP>
__device__ double ros_attempt(const DevMech &m, const Opts &o, double *lds, double *F, double y, double p,
                              const double *dlnA, int lane, double hc, double *err, double *dinv_out = nullptr)
{
    const int n = m.N + 1;
    double *U = lds + Lds<NP>::U;
    RowCoef rc;
    const double f0 = rhs_jac<NP>(m, lds, y, p, dlnA, lane, rc);
    const double dinv = factor_matrix<NP>(m, lds, rc, lane, 1.0 / (GAM * hc), F);
    if (dinv_out) *dinv_out = dinv;
    const double ih = 1.0 / hc;
    double flast = f0;
#pragma unroll 1
    for (int i = 0; i < NS; ++i) {
        double fi;
        const int reuse = TREUSE[i];
        if (reuse == 0) {
            fi = f0;
        } else if (reuse > 0) {
            fi = flast;  // the stage it names is the last one evaluated
        } else {
            double ys = y;
            for (int j = 0; j < i; ++j) ys += TA[i][j] * U[j * WAVE + lane];
            fi = rhs<NP>(m, lds, ys, p, dlnA, lane);
            flast = fi;
        }
        for (int j = 0; j < i; ++j) fi += (TC[i][j] * ih) * U[j * WAVE + lane];
        if (lane >= n) fi = 0.0;
        U[i * WAVE + lane] = lu_solve<NP>(F, dinv, fi, lane);
    }
    double ynew = y, ev = 0.0;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const double ui = U[i * WAVE + lane];
        ynew += TM[i] * ui;
        ev += TE[i] * ui;
    }
    double e2 = 0.0;
    if (lane < n) {
        const double sc = o.atol + o.rtol * fmax(fabs(y), fabs(ynew));
        const double r = ev / sc;
        e2 = r * r;
    }
    *err = sqrt(wave_sum(e2) / n);
    return ynew;
}

// One step of the extrapolation baseline: the linearly implicit Euler method
//   (I - h J(y0)) (y_{i+1} - y_i) = h f(y_i),  h = H / n_j,
// on the step numbers n_j = j (j = 1..EXK), each column's end state T_{j,1}
// extrapolated to h -> 0 by Aitken-Neville for an expansion in powers of h,
//   T_{j,l+1} = T_{j,l} + (T_{j,l} - T_{j-1,l}) (j - l) / l.
// T_{EXK,EXK} is the new state (order EXK); T_{EXK,EXK} - T_{EXK,EXK-1} the
// error estimate (order EXK - 1 local error, so the controller's
// err^(-1/4) matches EXK = 4).  The LDS term region holds one matrix, so
// each column recomputes J(y0) before factorising I/h - J (the same
// Jacobian: the pass is deterministic).  Row j of the tableau overwrites
// row j - 1 in the stage-vector area U.
constexpr int EXK = 4;
template <int NP>
__device__ double extrap_attempt(const DevMech &m, const Opts &o, double *lds, double y, double p,
                                 const double *dlnA, int lane, double H, double *err)
{
    const int n = m.N + 1;
    double *U = lds + Lds<NP>::U;
    double *F = lds + Lds<NP>::P;
    double tkk = y, tk1 = y;
#pragma unroll 1
    for (int j = 1; j <= EXK; ++j) {
        RowCoef rc;
        const double f0 = rhs_jac<NP>(m, lds, y, p, dlnA, lane, rc);
        const double h = H / j;
        const double dinv = factor_matrix<NP>(m, lds, rc, lane, 1.0 / h, F);
        double yi = y, fi = f0;
#pragma unroll 1
        for (int i = 0; i < j; ++i) {
            if (i > 0) fi = rhs<NP>(m, lds, yi, p, dlnA, lane);
            if (lane >= n) fi = 0.0;
            yi += lu_solve<NP>(F, dinv, fi, lane);
        }
        // row j of the tableau from row j - 1 (U[l-1] holds T_{j-1,l})
        double t = yi;
#pragma unroll 1
        for (int l = 1; l < j; ++l) {
            const double told = U[(l - 1) * WAVE + lane];
            const double next = t + (t - told) * ((double)(j - l) / (double)l);
            U[(l - 1) * WAVE + lane] = t;
            t = next;
        }
        U[(j - 1) * WAVE + lane] = t;
        if (j == EXK) {
            tkk = t;
            tk1 = U[(EXK - 2) * WAVE + lane];
        }
    }
    double e2 = 0.0;
    if (lane < n) {
        const double sc = o.atol + o.rtol * fmax(fabs(y), fabs(tkk));
        const double r = (tkk - tk1) / sc;
        e2 = r * r;
    }
    *err = sqrt(wave_sum(e2) / n);
    return lane < n ? tkk : 0.0;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
__device__ __forceinline__ double load_state(const DevMech &m, const double *T, const double *Y, int64_t ld,
                                             int64_t c, int lane)
{
    if (lane < m.N) return Y[(int64_t)lane * ld + c];
    if (lane == m.N) return T[c];
    return 0.0;
}

// ---------------------------------------------------------------------------
// step-size controller
// ---------------------------------------------------------------------------
// Controller state of one cell.
struct Ctl {
    double t, h, hnext;
    int nacc, nrej, nonfinite;
    bool last_rej;
};

__device__ __forceinline__ Ctl ctl_init(double h, double dt) { return Ctl{0.0, h, dt, 0, 0, 0, false}; }

// Size of the next attempt.  Returns SC_CELL_OK (hc and last set) or the
// status that ends the cell.
__device__ __forceinline__ int ctl_begin(const Ctl &s, const Opts &o, double dt, double &hc, bool &last)
{
    if (s.nacc + s.nrej >= o.max_steps) return SC_CELL_MAX_STEPS;
    if (s.h < 1e-20 * dt) return SC_CELL_H_UNDERFLOW;
    last = false;
    hc = o.hmax_frac > 0.0 ? fmin(s.h, o.hmax_frac * dt) : s.h;
    if (s.t + hc >= dt) {
        hc = dt - s.t;
        last = true;
    }
    return SC_CELL_OK;
}

// Decision on an attempt of size hc with scaled error err: 1 accepted,
// 0 rejected, or minus the status that ends the cell.  Adaptive mode: new
// step 0.9 err^(-1/4) clamped to [0.2, 6] (no growth right after a
// rejection); five non-finite estimates in a row give up.  Fixed mode: every
// finite attempt is accepted and h stays.
__device__ __forceinline__ int ctl_end(Ctl &s, const Opts &o, double err, double hc, bool last, double dt)
{
    if (o.fixed) {
        if (!isfinite(err)) return -SC_CELL_NONFINITE;
        ++s.nacc;
        s.t = last ? dt : s.t + hc;
        s.hnext = s.h;
        return 1;
    }
    if (!isfinite(err)) {
        ++s.nrej;
        s.h = hc * 0.2;
        s.last_rej = true;
        if (++s.nonfinite >= 5) return -SC_CELL_NONFINITE;
        return 0;
    }
    s.nonfinite = 0;
    // err^(-1/4) as two correctly rounded square roots: no library pow,
    // whose simplification depends on the surrounding code, so every
    // kernel that runs the controller takes the same steps
    double fac = 0.9 / sqrt(sqrt(fmax(err, 1e-300)));
    fac = fmin(6.0, fmax(0.2, fac));
    if (err <= 1.0) {
        ++s.nacc;
        s.t = last ? dt : s.t + hc;
        if (s.last_rej) fac = fmin(fac, 1.0);
        s.last_rej = false;
        s.h = hc * fac;
        s.hnext = s.h;
        return 1;
    }
    ++s.nrej;
    s.last_rej = true;
    s.h = hc * fmin(fac, 1.0);
    return 0;
}

// Integrate one cell's state y over [0, dt] (dt > 0) from the initial step
// h: error-controlled (or fixed) steps of the method METH (SC_METHOD_*).
// Returns the cell status; the controller state (step counts, proposed
// next step) is left in s.
template <int NP, int METH = SC_METHOD_ROS4>
__device__ int advance(const DevMech &m, const Opts &o, double *lds, double &y, double p, double dt,
                       const double *dlnA, int lane, Ctl &s)
{
#pragma unroll 1
    while (true) {
        double hc;
        bool last;
        const int st = ctl_begin(s, o, dt, hc, last);
        if (st != SC_CELL_OK) return st;
        double err;
        double ynew;
        if constexpr (METH == SC_METHOD_EXTRAP)
            ynew = extrap_attempt<NP>(m, o, lds, y, p, dlnA, lane, hc, &err);
        else
            ynew = ros_attempt<NP>(m, o, lds, lds + Lds<NP>::P, y, p, dlnA, lane, hc, &err);
        const int r = ctl_end(s, o, err, hc, last, dt);
        if (r < 0) return -r;
        if (r == 1) {
            y = ynew;
            if (last) return SC_CELL_OK;
        }
    }
}

// Validate a cell's inputs (uniform decision over the wave).
__device__ __forceinline__ bool bad_input(const DevMech &m, double y, double p, double dt, int lane)
{
    const int n = m.N + 1;
    const bool bad_lane = lane < n && !isfinite(y);
    const double T = rdlane(y, m.N);
    return __any(bad_lane) || !(T > 0.0) || !isfinite(T) || !(p > 0.0) || !isfinite(p) || !(dt >= 0.0) ||
           !isfinite(dt);
}

// Initial step: dt, or the caller's h when positive and finite (capped at dt).
__device__ __forceinline__ double initial_step(const double *h_io, int64_t c, double dt)
{
    double h = dt;
    if (h_io) {
        const double h0 = h_io[c];
        if (h0 > 0.0 && isfinite(h0)) h = fmin(h0, dt);
    }
    return h;
}
}  // namespace scdev
