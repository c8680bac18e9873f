// Device kernels for batched constant-pressure reactor integration (gfx950).
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
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include <hipcub/hipcub.hpp>

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
__constant__ double TA[NS][NS] = {{0.0, 0.0, 0.0, 0.0},
                                  {1.0474566606950075, 0.0, 0.0, 0.0},
                                  {1.5266834054578882, 0.49110997987229194, 0.0, 0.0},
                                  {1.5266834054578882, 0.49110997987229194, 0.0, 0.0}};
__constant__ double TC[NS][NS] = {{0.0, 0.0, 0.0, 0.0},
                                  {-2.8287104387961546, 0.0, 0.0, 0.0},
                                  {-1.1423273772481277, 0.9544101947030211, 0.0, 0.0},
                                  {-3.972521690537523, -0.6901523982223108, -1.548869644699513, 0.0}};
__constant__ double TM[NS] = {2.326763557172835, -0.7953731300411474, 1.6632540048577067, 1.0474566606950075};
__constant__ double TE[NS] = {0.4092508278871161, -1.0795845833425672, 0.9649495643943683,
                              1.0474566606950078};  // m - mhat
// function value of a stage: 0 = f(y) from the Jacobian pass, -1 = evaluate,
// k > 0 = reuse the value evaluated at stage k (same point)
__constant__ int TREUSE[NS] = {0, -1, -1, 2};
constexpr double ERR_EXP = 1.0 / 4.0;  // 1/(embedded order + 1)

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
// LDS layout of one cell (doubles)
// ---------------------------------------------------------------------------
template <int NP>
struct Lds {
    static constexpr int P = 0;          // NP x NP Jacobian terms, later the LU factors
    static constexpr int C = NP * NP;    // concentrations
    static constexpr int G = C + NP;     // g/RT
    static constexpr int H = G + NP;     // h/RT
    static constexpr int WD = H + NP;    // production-rate accumulator
    static constexpr int UA = WD + NP;   // Euler-term accumulator
    static constexpr int IW = UA + NP;   // 1/W_c (0 for c >= N)
    static constexpr int U = IW + NP;    // NS stage vectors, WAVE apart
    static constexpr int SIZE = U + NS * WAVE;
};

// Per-cell uniform quantities at the point where a right-hand side was taken.
struct Mix {
    double T, invT, lnT, p, rho, Wbar, cp;
};

struct Thermo {
    double cpR, hRT, sR, dcpR;
};

// NASA-7 of species k (single temperature range)
__device__ __forceinline__ Thermo nasa7(const DevMech &m, int k, double T, double lnT, double invT)
{
    const int N = m.N;
    const double *a = m.nasa();
    const double a0 = a[k], a1 = a[N + k], a2 = a[2 * N + k], a3 = a[3 * N + k], a4 = a[4 * N + k],
                 a5 = a[5 * N + k], a6 = a[6 * N + k];
    Thermo t;
    t.cpR = a0 + T * (a1 + T * (a2 + T * (a3 + T * a4)));
    t.hRT = a0 + T * (a1 * 0.5 + T * (a2 * (1.0 / 3.0) + T * (a3 * 0.25 + T * a4 * 0.2))) + a5 * invT;
    t.sR = a0 * lnT + T * (a1 + T * (a2 * 0.5 + T * (a3 * (1.0 / 3.0) + T * a4 * 0.25))) + a6;
    t.dcpR = a1 + T * (2.0 * a2 + T * (3.0 * a3 + T * 4.0 * a4));
    return t;
}

// Mixture state from the lane-distributed y (lane k < N: Y_k, lane N: T);
// writes C, g/RT, h/RT to LDS and clears the accumulators.
template <int NP>
__device__ __forceinline__ Mix mixture(const DevMech &m, double *lds, double y, double p, Thermo &th, int lane)
{
    const int N = m.N;
    Mix x;
    x.T = rdlane(y, N);
    x.invT = 1.0 / x.T;
    x.lnT = log(x.T);
    x.p = p;
    double yw = 0.0, cpw = 0.0;
    th = Thermo{0, 0, 0, 0};
    if (lane < N) {
        th = nasa7(m, lane, x.T, x.lnT, x.invT);
        yw = y * m.invW()[lane];
        cpw = th.cpR * yw;
    }
    x.Wbar = 1.0 / wave_sum(yw);
    x.rho = p * x.Wbar * x.invT / m.Rgas;
    x.cp = m.Rgas * wave_sum(cpw);
    if (lane < N) {
        lds[Lds<NP>::C + lane] = x.rho * yw;
        lds[Lds<NP>::G + lane] = th.hRT - th.sR;
        lds[Lds<NP>::H + lane] = th.hRT;
        lds[Lds<NP>::WD + lane] = 0.0;
        lds[Lds<NP>::UA + lane] = 0.0;
    }
    return x;
}

__device__ __forceinline__ double ipow(double c, int nu)
{
    double r = c;
    if (nu >= 2) r *= c;
    if (nu >= 3) r *= c;
    return r;
}
__device__ __forceinline__ double dipow(double c, int nu)  // d(c^nu)/dc
{
    return nu == 1 ? 1.0 : nu == 2 ? 2.0 * c : 3.0 * c * c;
}

// One reaction's rate of progress and, in the Jacobian pass, its derivatives
// with respect to the slot species' concentrations and to T.  Slots: 0..2
// reactants, 3..5 products, 6..9 enhanced third-body species.
struct RxOut {
    double q;             // net rate of progress (mol/m^3/s)
    double d[sc::NDEP];   // dq/dC of slot species
    double dT;            // dq/dT at fixed C
    double euler;         // q - sum_s C_s dq/dC_s
    double dH;            // reaction enthalpy / RT
};

template <bool JAC>
__device__ __forceinline__ RxOut reaction(const DevMech &m, const double *lds, int j, const Mix &x, double dl,
                                          int CO, int GO, int HO)
{
    const RxRec &rr = m.rx[j];
    const int kind = rr.kind;
    const int nr = rr.nr, np = rr.np;
    const double lnkinf = rr.lnA + dl + rr.b * x.lnT - rr.EaR * x.invT;
    const double kinf = exp(lnkinf);
    int rn[sc::MAXSIDE], pn[sc::MAXSIDE];
    double rc[sc::MAXSIDE], pc[sc::MAXSIDE];
    double dG = 0.0, dH = 0.0;
#pragma unroll
    for (int i = 0; i < sc::MAXSIDE; ++i) {
        const bool ur = i < nr, up = i < np;
        const int rs = ur ? rr.rsp[i] : 0;
        const int ps = up ? rr.psp[i] : 0;
        rn[i] = ur ? rr.rnu[i] : 0;
        pn[i] = up ? rr.pnu[i] : 0;
        rc[i] = ur ? lds[CO + rs] : 1.0;
        pc[i] = up ? lds[CO + ps] : 1.0;
        dG += pn[i] * (up ? lds[GO + ps] : 0.0) - rn[i] * (ur ? lds[GO + rs] : 0.0);
        if (JAC) dH += pn[i] * (up ? lds[HO + ps] : 0.0) - rn[i] * (ur ? lds[HO + rs] : 0.0);
    }
    const int dnu = rr.dnu;
    const double lnKc = -dG + dnu * (m.lnp0R - x.lnT);
    // third-body concentration, rewritten with sum_k C_k = p/(R T):
    // [M] = p/(RT) + sum_enhanced (alpha - 1) C
    double M = 0.0;
    const int ne = rr.neff;
    double ec[sc::MAXENH], ea[sc::MAXENH];
#pragma unroll
    for (int e = 0; e < sc::MAXENH; ++e) {
        const bool ue = e < ne;
        ea[e] = ue ? rr.eam1[e] : 0.0;
        ec[e] = ue ? lds[CO + rr.esp[e]] : 0.0;
    }
    if (kind != sc::RX_PLAIN) {
        M = x.p * x.invT / m.Rgas;
#pragma unroll
        for (int e = 0; e < sc::MAXENH; ++e) M += ea[e] * ec[e];
    }
    double kf = kinf, phi = 0.0, dlnF_T = 0.0, dlnk0 = 0.0;
    if (kind == sc::RX_TROE) {
        const TroeRec &tr = m.troe[rr.tix];
        const double lnk0 = tr.lnA0 + dl + tr.b0 * x.lnT - tr.Ea0R * x.invT;
        const double Pr = exp(lnk0 - lnkinf) * M;
        const double a = tr.a, iT3 = tr.iT3, iT1 = tr.iT1, T2 = tr.T2;
        const double e3 = exp(-x.T * iT3), e1 = exp(-x.T * iT1), e2 = exp(-T2 * x.invT);
        const double Fc = (1.0 - a) * e3 + a * e1 + e2;
        const double L = log10(Fc);
        const double cc = -0.4 - 0.67 * L, nn = 0.75 - 1.27 * L;
        const double X = log10(Pr) + cc;
        const double D = nn - 0.14 * X;
        const double f = X / D;
        const double opf = 1.0 + f * f;
        const double lF = L / opf;
        kf = kinf * (Pr / (1.0 + Pr)) * exp(2.302585092994046 * lF);
        if (JAC) {
            const double g = -L * 2.0 * f / (opf * opf);
            phi = 1.0 / (1.0 + Pr) + g * (nn / (D * D));  // dln kf / dln Pr
            const double dlF_dL = 1.0 / opf + g * ((-0.67 * nn + 1.27 * X) / (D * D));
            const double dFc = -(1.0 - a) * iT3 * e3 - a * iT1 * e1 + T2 * x.invT * x.invT * e2;
            dlnF_T = dlF_dL * dFc / Fc;  // dln F/dT at fixed Pr
            dlnk0 = (tr.b0 + tr.Ea0R * x.invT) * x.invT;
        }
    }
    const double kr = kf * exp(-lnKc);
    const double p0 = ipow(rc[0], rn[0]), p1 = ipow(rc[1], rn[1]), p2 = ipow(rc[2], rn[2]);
    const double s0 = ipow(pc[0], pn[0]), s1 = ipow(pc[1], pn[1]), s2 = ipow(pc[2], pn[2]);
    const double Rf = kf * (p0 * p1 * p2), Rr = kr * (s0 * s1 * s2);
    const double q0 = Rf - Rr;
    RxOut o;
    o.q = kind == sc::RX_THIRD ? q0 * M : q0;
    if (!JAC) return o;
    const double fsc = kind == sc::RX_THIRD ? M : 1.0;
    o.d[0] = nr > 0 ? fsc * kf * dipow(rc[0], rn[0]) * p1 * p2 : 0.0;
    o.d[1] = nr > 1 ? fsc * kf * dipow(rc[1], rn[1]) * p0 * p2 : 0.0;
    o.d[2] = nr > 2 ? fsc * kf * dipow(rc[2], rn[2]) * p0 * p1 : 0.0;
    o.d[3] = np > 0 ? -fsc * kr * dipow(pc[0], pn[0]) * s1 * s2 : 0.0;
    o.d[4] = np > 1 ? -fsc * kr * dipow(pc[1], pn[1]) * s0 * s2 : 0.0;
    o.d[5] = np > 2 ? -fsc * kr * dipow(pc[2], pn[2]) * s0 * s1 : 0.0;
    const double dlnkinf = (rr.b + rr.EaR * x.invT) * x.invT;
    const double dlnKc = (dH - dnu) * x.invT;
    const double dMdT = -x.p * x.invT * x.invT / m.Rgas;
    double dqM = 0.0;  // dq/d[M]
    double dlnkf = dlnkinf;
    if (kind == sc::RX_THIRD) {
        dqM = q0;
    } else if (kind == sc::RX_TROE) {
        dqM = q0 * phi / M;
        dlnkf = dlnkinf + phi * (dlnk0 - dlnkinf + dMdT / M) + dlnF_T;
    }
    double dT = q0 * dlnkf + Rr * dlnKc;
    if (kind == sc::RX_THIRD) dT = M * dT + q0 * dMdT;
#pragma unroll
    for (int e = 0; e < sc::MAXENH; ++e) o.d[6 + e] = dqM * ea[e];
    o.dT = dT;
    double eu = o.q;
#pragma unroll
    for (int i = 0; i < sc::MAXSIDE; ++i)
        eu -= (i < nr ? rc[i] : 0.0) * o.d[i] + (i < np ? pc[i] : 0.0) * o.d[3 + i];
#pragma unroll
    for (int e = 0; e < sc::MAXENH; ++e) eu -= ec[e] * o.d[6 + e];
    o.euler = eu;
    o.dH = dH;
    return o;
}

// Scatter a reaction's contributions: production rates (always) and, in the
// Jacobian pass, the sparse analytical terms of every (row, slot) pair, the
// temperature column and (weighted by the reaction enthalpy) the temperature row.
template <int NP, bool JAC>
__device__ __forceinline__ void scatter(const DevMech &m, double *lds, int j, const RxOut &o, double dHJ)
{
    const int N = m.N;
    const RxRec &rr = m.rx[j];
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
    // rows: reactants then products (a rolled loop keeps one row's terms live)
#pragma unroll 1
    for (int r = 0; r < nr + np; ++r) {
        const bool isr = r < nr;
        const int ri = isr ? r : r - nr;
        const int row = isr ? rr.rsp[ri] : rr.psp[ri];
        const double nu = isr ? -(double)rr.rnu[ri] : (double)rr.pnu[ri];
        atomicAdd(&lds[Lds<NP>::WD + row], nu * o.q);
        if (JAC) {
            atomicAdd(&lds[Lds<NP>::UA + row], nu * o.euler);
            double *Prow = P + row * NP;
#pragma unroll
            for (int s = 0; s < sc::NDEP; ++s)
                if (use[s]) atomicAdd(&Prow[col[s]], nu * o.d[s]);
            atomicAdd(&Prow[N], nu * o.dT);
        }
    }
    if (JAC) {
#pragma unroll
        for (int s = 0; s < sc::NDEP; ++s)
            if (use[s]) atomicAdd(&P[N * NP + col[s]], dHJ * o.d[s]);
        atomicAdd(&P[N * NP + N], dHJ * o.dT);
    }
}

// Right-hand side f(y), lane-distributed (0 in padding lanes).
template <int NP>
__device__ double rhs(const DevMech &m, double *lds, double y, double p, const double *dlnA, int lane)
{
    const int N = m.N, R = m.R;
    Thermo th;
    const Mix x = mixture<NP>(m, lds, y, p, th, lane);
    wave_sync();
#pragma unroll 1
    for (int j = lane; j < R; j += WAVE) {
        const double dl = dlnA ? dlnA[m.rx[j].orig] : 0.0;
        const RxOut o = reaction<false>(m, lds, j, x, dl, Lds<NP>::C, Lds<NP>::G, Lds<NP>::H);
        scatter<NP, false>(m, lds, j, o, 0.0);
    }
    wave_sync();
    double f = 0.0, hw = 0.0;
    if (lane < N) {
        const double wd = lds[Lds<NP>::WD + lane];
        f = m.W()[lane] * wd / x.rho;
        hw = th.hRT * wd;
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

// Jacobian pass: f(y) plus the analytical terms, finalised in LDS.  With
// Q != nullptr the rates of progress q_j are kept there (execution order),
// for the parameter part of vector-Jacobian products.
template <int NP>
__device__ double rhs_jac(const DevMech &m, double *lds, double y, double p, const double *dlnA, int lane,
                          RowCoef &rc, double *Q = nullptr, Mix *xout = nullptr)
{
    const int N = m.N, R = m.R;
    double *P = lds + Lds<NP>::P;
    Thermo th;
    const Mix x = mixture<NP>(m, lds, y, p, th, lane);
    if (lane < NP) {
#pragma unroll 4
        for (int i = 0; i < NP; ++i) P[i * NP + lane] = 0.0;  // lane c clears column c
    }
    wave_sync();
    const double RT = m.Rgas * x.T;
#pragma unroll 1
    for (int j = lane; j < R; j += WAVE) {
        const double dl = dlnA ? dlnA[m.rx[j].orig] : 0.0;
        const RxOut o = reaction<true>(m, lds, j, x, dl, Lds<NP>::C, Lds<NP>::G, Lds<NP>::H);
        scatter<NP, true>(m, lds, j, o, o.dH * RT);
        if (Q) Q[j] = o.q;
    }
    wave_sync();
    double f = 0.0, hw = 0.0, eu = 0.0, cpf = 0.0, dcp = 0.0, uk = 0.0, Wk = 0.0;
    if (lane < N) {
        Wk = m.W()[lane];
        const double iw = m.invW()[lane];
        const double wd = lds[Lds<NP>::WD + lane];
        f = Wk * wd / x.rho;
        uk = Wk * lds[Lds<NP>::UA + lane] / x.rho;
        hw = th.hRT * wd;
        eu = th.hRT * uk * iw;   // (h_k/(R T W_k)) u_k
        cpf = th.cpR * f * iw;   // cp_k/(R W_k) f_k
        dcp = th.dcpR * y * iw;  // dcp_k/dT/(R W_k) Y_k
    }
    const double H = RT * wave_sum(hw);
    const double Eu = RT * wave_sum(eu);  // sum_k (h_k/W_k) u_k
    const double Scpf = m.Rgas * wave_sum(cpf);
    const double Sdcp = m.Rgas * wave_sum(dcp);
    const double fT = -H / (x.rho * x.cp);
    if (lane == N) f = fT;
    // fold the column-dependent parts of the temperature row into P[N][*]:
    // J_Tm = -(1/cp) (1/W_m) (P_Tm + Wbar Eu + fT cp_m),
    // J_TT = -(1/cp) (P_TT/rho + Eu/T + sum cp_k f_k/W_k + fT sum dcp_k Y_k/W_k)
    if (lane < N) P[N * NP + lane] += x.Wbar * Eu + fT * m.Rgas * th.cpR;
    if (lane == N) P[N * NP + N] = P[N * NP + N] / x.rho + Eu * x.invT + Scpf + fT * Sdcp;
    if (lane < NP) lds[Lds<NP>::IW + lane] = lane < N ? m.invW()[lane] : 0.0;
    wave_sync();
    const double invcp = 1.0 / x.cp;
    if (lane < N) {
        // species rows: J_km = (W_k/W_m) P_km + u_k Wbar/W_m, J_kT = (W_k/rho) P_kT + u_k/T
        rc = RowCoef{Wk, uk * x.Wbar, Wk / x.rho, uk * x.invT};
    } else if (lane == N) {
        rc = RowCoef{-invcp, 0.0, -invcp, 0.0};
    } else {
        rc = RowCoef{0.0, 0.0, 0.0, 0.0};
    }
    if (xout) *xout = x;
    return f;
}

// Row `lane` of J from the finalised LDS terms into registers.
template <int NP>
__device__ __forceinline__ void jac_row(const DevMech &m, const double *lds, const RowCoef &rc, int lane,
                                        double (&a)[NP])
{
    const int N = m.N;
    const double *P = lds + Lds<NP>::P + (lane < NP ? lane : 0) * NP;
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

// Park the factors in LDS, column-major (F[c*NP + i] = row i, column c), so
// that every read in the triangular solves is one conflict-free wave access.
template <int NP>
__device__ __forceinline__ void store_factors(double *F, const double (&a)[NP], int lane)
{
    if (lane < NP) {
#pragma unroll
        for (int c = 0; c < NP; ++c) {
            F[c * NP + lane] = a[c];
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
        const double l = F[k * NP + li];
        const double z = rdlane(b, k);
        if (lane > k) b = fma(-l, z, b);
        SC_FENCE_EVERY(k);
    }
#pragma unroll
    for (int k = NP - 1; k >= 0; --k) {
        if (lane == k) b *= dinv;
        const double z = rdlane(b, k);
        const double u = F[k * NP + li];
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
                              const double *dlnA, int lane, double hc, double *err)
{
    const int n = m.N + 1;
    double *U = lds + Lds<NP>::U;
    RowCoef rc;
    const double f0 = rhs_jac<NP>(m, lds, y, p, dlnA, lane, rc);
    const double dinv = factor_matrix<NP>(m, lds, rc, lane, 1.0 / (GAM * hc), F);
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

template <int NP>
__global__ void __launch_bounds__(WAVE) k_rhs(DevMech m, int64_t n, const double *T, const double *p,
                                              const double *Y, int64_t ld, const double *dlnA, double *fT,
                                              double *fY)
{
    extern __shared__ double lds[];
    const int lane = threadIdx.x;
    const int64_t c = blockIdx.x;
    if (c >= n) return;
    const double y = load_state(m, T, Y, ld, c, lane);
    const double f = rhs<NP>(m, lds, y, p[c], dlnA, lane);
    if (lane < m.N) fY[(int64_t)lane * ld + c] = f;
    if (lane == m.N) fT[c] = f;
}

template <int NP>
__global__ void __launch_bounds__(WAVE) k_jac(DevMech m, int64_t n, const double *T, const double *p,
                                              const double *Y, int64_t ld, const double *dlnA, double *J)
{
    extern __shared__ double lds[];
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

template <int NP>
__global__ void __launch_bounds__(WAVE) k_linsolve(DevMech m, int64_t n, const double *T, const double *p,
                                                   const double *Y, int64_t ld, const double *dlnA,
                                                   const double *hg, const double *b, double *x)
{
    extern __shared__ double lds[];
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

// One cell over [0, dt] with the Rosenbrock method and error control.
template <int NP>
__device__ void integrate_cell(const DevMech &m, const Opts &o, double *lds, int64_t c, int lane, const double *T0,
                               const double *P, const double *Y0, int64_t ld, const double *DT, const double *dlnA,
                               double *h_io, double *T1, double *Y1, int32_t *status, int32_t *nacc_out,
                               int32_t *nrej_out)
{
    const int N = m.N, n = N + 1;
    double y = load_state(m, T0, Y0, ld, c, lane);
    const double p = P[c], dt = DT[c];
    // input validation (uniform decision)
    const bool bad_lane = lane < n && !isfinite(y);
    const double T = rdlane(y, N);
    const bool bad = __any(bad_lane) || !(T > 0.0) || !isfinite(T) || !(p > 0.0) || !isfinite(p) ||
                     !(dt >= 0.0) || !isfinite(dt);
    int st = SC_CELL_OK, nacc = 0, nrej = 0;
    double hnext = dt;
    if (bad) {
        st = SC_CELL_BAD_INPUT;
    } else if (dt > 0.0) {
        double h = dt;
        if (h_io) {
            const double h0 = h_io[c];
            if (h0 > 0.0 && isfinite(h0)) h = fmin(h0, dt);
        }
        double t = 0.0;
        bool last_rej = false;
        int nonfinite = 0;
#pragma unroll 1
        while (true) {
            if (nacc + nrej >= o.max_steps) { st = SC_CELL_MAX_STEPS; break; }
            if (h < 1e-20 * dt) { st = SC_CELL_H_UNDERFLOW; break; }
            // Jacobian terms at y (recomputed after a rejection too: their LDS
            // region holds the LU factors while the stages run)
            bool last = false;
            double hc = h;
            if (t + hc >= dt) { hc = dt - t; last = true; }
            double err;
            const double ynew = ros_attempt<NP>(m, o, lds, lds + Lds<NP>::P, y, p, dlnA, lane, hc, &err);
            if (!isfinite(err)) {
                ++nrej;
                h = hc * 0.2;
                last_rej = true;
                if (++nonfinite >= 5) { st = SC_CELL_NONFINITE; break; }
                continue;
            }
            nonfinite = 0;
            double fac = 0.9 * pow(fmax(err, 1e-300), -ERR_EXP);
            fac = fmin(6.0, fmax(0.2, fac));
            if (err <= 1.0) {
                ++nacc;
                y = ynew;
                t = last ? dt : t + hc;
                if (last_rej) fac = fmin(fac, 1.0);
                last_rej = false;
                h = hc * fac;
                hnext = h;
                if (last) break;
            } else {
                ++nrej;
                last_rej = true;
                h = hc * fmin(fac, 1.0);
            }
        }
    }
    if (lane < N) Y1[(int64_t)lane * ld + c] = y;
    if (lane == N) {
        T1[c] = y;
        status[c] = st;
        if (nacc_out) nacc_out[c] = nacc;
        if (nrej_out) nrej_out[c] = nrej;
        if (h_io && st == SC_CELL_OK && dt > 0.0) h_io[c] = hnext;
    }
}

template <int NP>
__global__ void __launch_bounds__(WAVE) k_integrate(DevMech m, Opts o, int64_t n, const double *T0, const double *P,
                                                    const double *Y0, int64_t ld, const double *DT,
                                                    const double *dlnA, double *h_io, double *T1, double *Y1,
                                                    int32_t *status, int32_t *nacc, int32_t *nrej)
{
    extern __shared__ double lds[];
    const int64_t c = blockIdx.x;
    if (c >= n) return;
    integrate_cell<NP>(m, o, lds, c, threadIdx.x, T0, P, Y0, ld, DT, dlnA, h_io, T1, Y1, status, nacc, nrej);
}

// Persistent variant: a resident grid; each wave pulls tiles of `tile` cells
// from a global counter (optionally through a permutation, e.g. longest dt
// first) until the queue is drained.  Per-cell arithmetic is identical to the
// plain kernel, so results are bitwise equal.
template <int NP>
__global__ void __launch_bounds__(WAVE) k_integrate_persistent(DevMech m, Opts o, int64_t n, const double *T0,
                                                               const double *P, const double *Y0, int64_t ld,
                                                               const double *DT, const double *dlnA, double *h_io,
                                                               double *T1, double *Y1, int32_t *status,
                                                               int32_t *nacc, int32_t *nrej,
                                                               unsigned long long *queue, const int32_t *perm,
                                                               int tile)
{
    extern __shared__ double lds[];
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
            integrate_cell<NP>(m, o, lds, c, lane, T0, P, Y0, ld, DT, dlnA, h_io, T1, Y1, status, nacc, nrej);
        }
    }
}

// Static mapping (the baseline the queue is compared with): workgroup w owns
// cells [w*group, (w+1)*group) and integrates them one after another.
template <int NP>
__global__ void __launch_bounds__(WAVE) k_integrate_static(DevMech m, Opts o, int64_t n, const double *T0,
                                                           const double *P, const double *Y0, int64_t ld,
                                                           const double *DT, const double *dlnA, double *h_io,
                                                           double *T1, double *Y1, int32_t *status, int32_t *nacc,
                                                           int32_t *nrej, int64_t group)
{
    extern __shared__ double lds[];
    const int64_t c0 = (int64_t)blockIdx.x * group;
    const int64_t c1 = min(c0 + group, n);
#pragma unroll 1
    for (int64_t c = c0; c < c1; ++c)
        integrate_cell<NP>(m, o, lds, c, threadIdx.x, T0, P, Y0, ld, DT, dlnA, h_io, T1, Y1, status, nacc, nrej);
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
    if (i < n) key[i] = na[i] + nr[i];
}

// ---------------------------------------------------------------------------
// launchers (host)
// ---------------------------------------------------------------------------
template <int NP>
size_t lds_bytes() { return sizeof(double) * Lds<NP>::SIZE; }

#define SC_DISPATCH(np, CALL)                         \
    switch (np) {                                     \
    case 16: { constexpr int NPV = 16; CALL; } break; \
    case 32: { constexpr int NPV = 32; CALL; } break; \
    case 56: { constexpr int NPV = 56; CALL; } break; \
    case 64: { constexpr int NPV = 64; CALL; } break; \
    default: return hipErrorInvalidValue;             \
    }

hipError_t launch_rhs(int np, const DevMech &m, int64_t n, const double *T, const double *p, const double *Y,
                      int64_t ld, const double *dlnA, double *fT, double *fY, hipStream_t s)
{
    SC_DISPATCH(np, hipLaunchKernelGGL(k_rhs<NPV>, dim3((unsigned)n), dim3(WAVE), lds_bytes<NPV>(), s, m, n, T, p,
                                       Y, ld, dlnA, fT, fY));
    return hipGetLastError();
}

hipError_t launch_jac(int np, const DevMech &m, int64_t n, const double *T, const double *p, const double *Y,
                      int64_t ld, const double *dlnA, double *J, hipStream_t s)
{
    SC_DISPATCH(np, hipLaunchKernelGGL(k_jac<NPV>, dim3((unsigned)n), dim3(WAVE), lds_bytes<NPV>(), s, m, n, T, p,
                                       Y, ld, dlnA, J));
    return hipGetLastError();
}

hipError_t launch_linsolve(int np, const DevMech &m, int64_t n, const double *T, const double *p, const double *Y,
                           int64_t ld, const double *dlnA, const double *hg, const double *b, double *x,
                           hipStream_t s)
{
    SC_DISPATCH(np, hipLaunchKernelGGL(k_linsolve<NPV>, dim3((unsigned)n), dim3(WAVE), lds_bytes<NPV>(), s, m, n,
                                       T, p, Y, ld, dlnA, hg, b, x));
    return hipGetLastError();
}

hipError_t launch_integrate(int np, const DevMech &m, const Opts &o, int64_t n, const double *T0, const double *p,
                            const double *Y0, int64_t ld, const double *dt, const double *dlnA, double *h_io,
                            double *T1, double *Y1, int32_t *st, int32_t *na, int32_t *nr, hipStream_t s)
{
    SC_DISPATCH(np, hipLaunchKernelGGL(k_integrate<NPV>, dim3((unsigned)n), dim3(WAVE), lds_bytes<NPV>(), s, m, o,
                                       n, T0, p, Y0, ld, dt, dlnA, h_io, T1, Y1, st, na, nr));
    return hipGetLastError();
}

hipError_t launch_integrate_persistent(int np, const DevMech &m, const Opts &o, int64_t n, const double *T0,
                                       const double *p, const double *Y0, int64_t ld, const double *dt,
                                       const double *dlnA, double *h_io, double *T1, double *Y1, int32_t *st,
                                       int32_t *na, int32_t *nr, unsigned long long *queue, const int32_t *perm,
                                       int tile, int grid, hipStream_t s)
{
    SC_DISPATCH(np, hipLaunchKernelGGL(k_integrate_persistent<NPV>, dim3((unsigned)grid), dim3(WAVE),
                                       lds_bytes<NPV>(), s, m, o, n, T0, p, Y0, ld, dt, dlnA, h_io, T1, Y1, st, na,
                                       nr, queue, perm, tile));
    return hipGetLastError();
}

hipError_t launch_integrate_static(int np, const DevMech &m, const Opts &o, int64_t n, const double *T0,
                                   const double *p, const double *Y0, int64_t ld, const double *dt,
                                   const double *dlnA, double *h_io, double *T1, double *Y1, int32_t *st,
                                   int32_t *na, int32_t *nr, int grid, hipStream_t s)
{
    const int64_t group = (n + grid - 1) / grid;
    const unsigned g = (unsigned)((n + group - 1) / group);
    SC_DISPATCH(np, hipLaunchKernelGGL(k_integrate_static<NPV>, dim3(g), dim3(WAVE), lds_bytes<NPV>(), s, m, o, n,
                                       T0, p, Y0, ld, dt, dlnA, h_io, T1, Y1, st, na, nr, group));
    return hipGetLastError();
}

// Cell permutation for the persistent queue: indices sorted by descending
// key (dt, or the previous call's step count), by a device radix sort.
// `ws` is grown on demand: [perm_in | perm_out | keys_out | cost keys | temp].
hipError_t order_cells(int order, int64_t n, const double *dt, const int32_t *na, const int32_t *nr,
                       void **ws, size_t *ws_bytes, int32_t **perm, hipStream_t s)
{
    const size_t al = 256;
    auto up = [&](size_t b) { return (b + al - 1) / al * al; };
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
    const size_t b_perm = up(sizeof(int32_t) * n), b_keys = up(sizeof(double) * n);
    const size_t need = 2 * b_perm + 2 * b_keys + up(tmp);
    if (*ws_bytes < need) {
        if (*ws) (void)hipFree(*ws);
        *ws = nullptr;
        *ws_bytes = 0;
        if ((e = hipMalloc(ws, need)) != hipSuccess) return e;
        *ws_bytes = need;
    }
    char *base = (char *)*ws;
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
    case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_integrate_persistent<16>, WAVE, lds_bytes<16>()); break;
    case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_integrate_persistent<32>, WAVE, lds_bytes<32>()); break;
    case 56: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_integrate_persistent<56>, WAVE, lds_bytes<56>()); break;
    case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_integrate_persistent<64>, WAVE, lds_bytes<64>()); break;
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
