// Discrete adjoint of the batched Rosenbrock integration (gfx950).
//
// The integrator maps (y0, dlnA) to y_S through S accepted steps
//   y_{n+1} = y_n + sum_i m_i u_i,   M u_i = f(Y_i) + sum_{j<i} (c_ij / h) u_j,
//   Y_i = y_n + sum_{j<i} a_ij u_j,  M = I/(gamma h) - J(y_n),
// with the step sizes h_n chosen by the controller.  The adjoint here is the
// exact derivative of that map with the step sequence frozen (the
// controller's decisions are not differentiated).  Per step, in reverse:
//   w_i = M^-T ubar_i (transposed solves with the step's own factors),
//   ubar_j += (c_ij / h) w_i + a_ij J(Y_i)^T fbar_i,
//   lambda_n = lambda_{n+1} + sum_points J(Y)^T fbar + sum_i d/dy (w_i . J(y_n) u_i),
// and every vector-Jacobian product also adds w . df/d(dlnA_j) to the
// per-reaction adjoint.  The second-derivative terms d/dy (w . J u) and
// their parameter parts are exact directional derivatives of the
// vector-Jacobian product along u_i, carried by dual numbers.
//
// One wavefront per cell, as in the forward kernels.  A resident grid pulls
// cells from a queue; each wave owns a slot of global scratch holding the
// accepted step sizes, up to NCK checkpointed states and one segment of
// recomputed states.  The recording forward pass stores every K-th state
// (K doubles, and every other checkpoint is dropped, when the slots fill);
// the reverse sweep walks the segments backwards, recomputing each segment's
// states from its checkpoint before reversing its steps.  Recording and
// replay run the same attempt routine as sc_integrate, so the recorded
// trajectory is the forward trajectory bit for bit.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "core.hpp"

namespace scdev {

// Checkpoint slots per cell (even).
constexpr int NCK = 2048;

// LDS of the adjoint: the forward layout followed by the vector-Jacobian
// product's work vectors, the per-stage adjoint vectors and the per-reaction
// parameter adjoint of the cell (R entries, execution order).
template <int NP>
struct LdsA {
    static constexpr int WW = Lds<NP>::SIZE;  // W_k w_k
    static constexpr int V = WW + NP;         // sum_j s_j dq_j/dC_m
    static constexpr int UB = V + NP;         // adjoints of the stage vectors
    static constexpr int WS = UB + NS * WAVE; // w_i = M^-T ubar_i
    static constexpr int FB = WS + NS * WAVE; // adjoints of the function values, by point
    static constexpr int TH = FB + NS * WAVE;
    static constexpr int fixed() { return TH; }
};


// g = J(y)^T w for the lane-distributed weight w (the Jacobian of sc_jacobian,
// built reaction by reaction without assembling it), and TH[j] += w . df/ddlnA_j
// = q_j s_j / rho.  With sigma_j = sum_k nu_kj W_k w_k and
// s_j = sigma_j - (w_T/cp) dH_j (dH_j the molar reaction enthalpy):
//   g_m = (1/W_m) [sum_j s_j dq_j/dC_m + Wbar B - (w_T/cp) f_T cp_m]   (m < N)
//   g_T = (1/rho) sum_j s_j dq_j/dT + B/T - (w_T/cp)(sum_k cp_k f_k/W_k + f_T sum_k Y_k dcp_k/dT/W_k)
// where B = (1/rho) sum_j s_j (q_j - sum_s C_s dq_j/dC_s) carries the
// density dependence of the concentrations.
// With S = Dual and y carrying a direction u (w fixed), the same arithmetic
// returns the exact directional derivative d/du (J(y)^T w) and adds
// d/du (q_j s_j / rho) to TH: the second-derivative terms of the adjoint.
// Dual passes keep their derivative arrays toff doubles from the values.
template <int NP, class S>
__device__ double vjp(const DevMech &m, double *lds, S y, double p, const double *dlnA, double w, int lane,
                      double *TH, int toff = 0)
{
    const int N = m.N, R = m.R;
    Thermo<S> th;
    const Mix<S> x = mixture<NP, S>(m, lds, y, p, th, lane, toff);
    double *WW = lds + LdsA<NP>::WW;
    const int V = LdsA<NP>::V;
    const S wc = rdlane(S(w), N) / x.cp;
    if (lane < N) {
        WW[lane] = m.W()[lane] * w;
        lds_put(lds, V + lane, S(0.0), toff);
    }
    wave_sync();
    const S RT = m.Rgas * x.T;
    const S irho = 1.0 / x.rho;
    S bacc = 0.0, tacc = 0.0;
#pragma unroll 1
    for (int j = lane; j < R; j += WAVE) {
        const RxRec rr = load_rec(m, j);
        const double dl = dlnA ? dlnA[rr.orig] : 0.0;
        const RxOut<S> o = reaction<true, S>(m, lds, rr, x, dl, Lds<NP>::C, Lds<NP>::G, Lds<NP>::H, toff);
        double sig = 0.0;
#pragma unroll
        for (int i = 0; i < sc::MAXSIDE; ++i) {
            if (i < rr.nr) sig -= rr.rnu[i] * WW[rr.rsp[i]];
            if (i < rr.np) sig += rr.pnu[i] * WW[rr.psp[i]];
        }
        const S s = sig - wc * (o.dH * RT);
        // production rates (for f_T) and V_m += s dq/dC_m over the slots
#pragma unroll
        for (int i = 0; i < sc::MAXSIDE; ++i) {
            if (i < rr.nr) {
                lds_add(lds, Lds<NP>::WD + rr.rsp[i], -(double)rr.rnu[i] * o.q, toff);
                lds_add(lds, V + rr.rsp[i], s * o.d[i], toff);
            }
            if (i < rr.np) {
                lds_add(lds, Lds<NP>::WD + rr.psp[i], (double)rr.pnu[i] * o.q, toff);
                lds_add(lds, V + rr.psp[i], s * o.d[3 + i], toff);
            }
        }
#pragma unroll
        for (int e = 0; e < sc::MAXENH; ++e)
            if (e < rr.neff) lds_add(lds, V + rr.esp[e], s * o.d[6 + e], toff);
        bacc += s * o.euler;
        tacc += s * o.dT;
        TH[j] += part(o.q * s * irho);
    }
    wave_sync();
    S hw = 0.0, cpf = 0.0, dcp = 0.0;
    if (lane < N) {
        const S wd = lds_get<S>(lds, Lds<NP>::WD + lane, toff);
        hw = th.hRT * wd;
        cpf = th.cpR * wd * irho;             // cp_k f_k / (R W_k)
        dcp = th.dcpR * y * m.invW()[lane];   // Y_k dcp_k/dT / (R W_k)
    }
    const S fT = -RT * wave_sum(hw) / (x.rho * x.cp);
    const S Scpf = m.Rgas * wave_sum(cpf);
    const S Sdcp = m.Rgas * wave_sum(dcp);
    const S B = wave_sum(bacc) * irho;
    const S A = wave_sum(tacc) * irho;
    S g = 0.0;
    if (lane < N) g = m.invW()[lane] * (lds_get<S>(lds, V + lane, toff) + x.Wbar * B - wc * fT * m.Rgas * th.cpR);
    if (lane == N) g = A + B * x.invT - wc * (Scpf + fT * Sdcp);
    wave_sync();
    return part(g);
}

// Solve (L U)^T x = b with the factors parked column-major in F: U^T z = b,
// then L^T x = z.  Each unknown is a dot product of one stored column with
// the solved part: one contiguous (conflict-free) LDS read per step and a
// wave reduction.
template <int NP>
__device__ double lu_solve_T(const double *F, double dinv, double b, int lane)
{
    constexpr int FS = Lds<NP>::PS;
    const int li = lane < NP ? lane : 0;
    double z = 0.0;
#pragma unroll 2
    for (int k = 0; k < NP; ++k) {
        const double u = F[k * FS + li];  // U_jk in lane j (j < k)
        const double s = wave_sum(lane < k ? u * z : 0.0);
        if (lane == k) z = (b - s) * dinv;
    }
    double x = 0.0;
#pragma unroll 2
    for (int k = NP - 1; k >= 0; --k) {
        const double l = F[k * FS + li];  // L_jk in lane j (j > k)
        const double s = wave_sum(lane > k ? l * x : 0.0);
        if (lane == k) x = z - s;
    }
    return lane < NP ? x : 0.0;
}

// Reverse one replayed step: the attempt from y with size hc has just left
// its stage vectors in U and its factors in F (dinv = 1/U_ii of this lane).
// Returns lambda_n from lambda_{n+1}; adds the parameter adjoint to TH.
template <int NP>
__device__ double step_adjoint(const DevMech &m, double *lds, double y, double p, const double *dlnA, int lane,
                               double hc, double dinv, double lam, double *TH)
{
    const int N = m.N, n = N + 1;
    const double *F = lds + Lds<NP>::P;
    const double *U = lds + Lds<NP>::U;
    double *UB = lds + LdsA<NP>::UB, *WS = lds + LdsA<NP>::WS, *FB = lds + LdsA<NP>::FB;
    const double ih = 1.0 / hc;
    // every lane touches only its own component of UB, WS and FB
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        UB[i * WAVE + lane] = TM[i] * lam;
        FB[i * WAVE + lane] = 0.0;
    }
    double lnew = lam;
#pragma unroll 1
    for (int i = NS - 1; i >= 0; --i) {
        const double w = lu_solve_T<NP>(F, dinv, lane < n ? UB[i * WAVE + lane] : 0.0, lane);
        WS[i * WAVE + lane] = w;
        for (int j = 0; j < i; ++j) UB[j * WAVE + lane] += (TC[i][j] * ih) * w;
        const int reuse = TREUSE[i];
        const int pt = reuse < 0 ? i : reuse;  // the stage whose point f was evaluated at
        FB[pt * WAVE + lane] += w;
        if (reuse < 0) {
            // this stage evaluated f at Y_i: its adjoint is complete (later
            // stages reusing the value were processed first)
            double ys = y;
            for (int j = 0; j < i; ++j) ys += TA[i][j] * U[j * WAVE + lane];
            const double g = vjp<NP, double>(m, lds, ys, p, dlnA, FB[i * WAVE + lane], lane, TH);
            for (int j = 0; j < i; ++j) UB[j * WAVE + lane] += TA[i][j] * g;
            lnew += g;
        }
    }
    // the dependence of M on y: sum_i d/dy (w_i . J(y) u_i) = sum_i d/du_i (J(y)^T w_i),
    // exact directional derivatives of the VJP along each stage vector (dual
    // numbers; the factors in the term region are no longer needed, so the
    // derivative arrays live there)
    const int toff = Lds<NP>::P - Lds<NP>::C;
    static_assert(LdsA<NP>::V + NP + (Lds<NP>::P - Lds<NP>::C) <= Lds<NP>::C,
                  "dual-pass derivative arrays must stay inside the term region");
#pragma unroll 1
    for (int i = 0; i < NS; ++i)
        lnew += vjp<NP, Dual>(m, lds, Dual(y, U[i * WAVE + lane]), p, dlnA, WS[i * WAVE + lane], lane, TH, toff);
    // f(y) itself: stage 0 and any stage reusing it
    lnew += vjp<NP, double>(m, lds, y, p, dlnA, FB[lane], lane, TH);
    return lnew;
}

// Accepted-step recorder of the forward pass (global scratch of this wave).
struct Recorder {
    double *H;   // step sizes, one per accepted step
    double *CK;  // NCK checkpoints, WAVE doubles each: state before step q*K
    int K;       // checkpoint stride (a power of two)

    __device__ __forceinline__ void accept(int q, double hc, double y, int lane)
    {
        if (lane == 0) H[q] = hc;
        if (q % K != 0) return;
        int i = q / K;
        if (i >= NCK) {
            // slots full (q = NCK K): keep the even ones, double the stride
#pragma unroll 1
            for (int s = 1; s < NCK / 2; ++s) CK[s * WAVE + lane] = CK[2 * s * WAVE + lane];
            K *= 2;
            i = q / K;
        }
        CK[i * WAVE + lane] = y;
    }
};

// Forward (recording) pass and reverse sweep of one cell.
template <int NP>
__device__ void adjoint_cell(const DevMech &m, const Opts &o, double *lds, int64_t c, int lane, const double *T0,
                             const double *P, const double *Y0, int64_t ld, const double *DT, const double *dlnA,
                             const double *h_in, const double *gT1, const double *gY1, double *gT0, double *gY0,
                             double *gcell, int64_t n_cells, int32_t *status, int32_t *nacc_out, double *T1,
                             double *Y1, double *slot, int hcap)
{
    const int N = m.N, R = m.R;
    double *TH = lds + LdsA<NP>::TH;
    double *F = lds + Lds<NP>::P;
#pragma unroll 1
    for (int j = lane; j < R; j += WAVE) TH[j] = 0.0;
    double y = load_state(m, T0, Y0, ld, c, lane);
    const double p = P[c], dt = DT[c];
    Ctl s = ctl_init(initial_step(h_in, c, dt), dt);
    Recorder rec{slot, slot + hcap, 1};
    double *SEG = rec.CK + NCK * WAVE;
    double lam = load_state(m, gT1, gY1, ld, c, lane);
    int st = SC_CELL_OK;

    enum { FWD, RECOMP, REV, DONE };
    int phase = FWD;
    if (bad_input(m, y, p, dt, lane)) {
        st = SC_CELL_BAD_INPUT;
        phase = DONE;
    } else if (!(dt > 0.0)) {
        phase = DONE;
    }
    // reverse-sweep position: segment seg covers steps [n0, n1); states
    // n0 < q < n1 are recomputed into SEG[q - n0 - 1]
    int seg = 0, n0 = 0, n1 = 0, q = 0;
    bool last = false;
    // one attempt per iteration, whatever the phase (one inlined copy of the
    // attempt routine)
#pragma unroll 1
    while (phase != DONE) {
        double ys, hc;
        if (phase == FWD) {
            st = ctl_begin(s, o, dt, hc, last);
            if (st != SC_CELL_OK) break;
            ys = y;
        } else {
            ys = q == n0 ? rec.CK[seg * WAVE + lane] : SEG[(q - n0 - 1) * WAVE + lane];
            hc = rec.H[q];
        }
        double err, dinv;
        const double ynew = ros_attempt<NP>(m, o, lds, F, ys, p, dlnA, lane, hc, &err, &dinv);
        if (phase == FWD) {
            const int r = ctl_end(s, o, err, hc, last, dt);
            if (r < 0) {
                st = -r;
                break;
            }
            if (r == 0) continue;
            rec.accept(s.nacc - 1, hc, y, lane);
            y = ynew;
            if (!last) continue;
            // forward done: outputs, then the reverse sweep from the last segment
            if (lane < N && Y1) Y1[(int64_t)lane * ld + c] = y;
            if (lane == N && T1) T1[c] = y;
            wave_sync();  // recorded step sizes visible to every lane
            seg = (s.nacc - 1) / rec.K;
            n0 = seg * rec.K;
            n1 = min(s.nacc, n0 + rec.K);
            q = n1 - n0 > 1 ? n0 : n1 - 1;
            phase = n1 - n0 > 1 ? RECOMP : REV;
        } else if (phase == RECOMP) {
            SEG[(q - n0) * WAVE + lane] = ynew;  // state q + 1
            ++q;
            if (q == n1 - 1) phase = REV;
        } else {
            lam = step_adjoint<NP>(m, lds, ys, p, dlnA, lane, hc, dinv, lam, TH);
            if (q > n0) {
                --q;
            } else if (seg > 0) {
                --seg;
                n0 = seg * rec.K;
                n1 = n0 + rec.K;
                q = rec.K > 1 ? n0 : n1 - 1;
                phase = rec.K > 1 ? RECOMP : REV;
            } else {
                phase = DONE;
            }
        }
    }
    const bool ok = st == SC_CELL_OK;
    if (!(dt > 0.0) && ok) {
        if (lane < N && Y1) Y1[(int64_t)lane * ld + c] = y;
        if (lane == N && T1) T1[c] = y;
    }
    if (!ok) {
        // no derivative of a failed integration
        lam = __longlong_as_double(0x7ff8000000000000ll);
        if (lane < N && Y1) Y1[(int64_t)lane * ld + c] = y;
        if (lane == N && T1) T1[c] = y;
    }
    if (lane < N) gY0[(int64_t)lane * ld + c] = lam;
    if (lane == N) {
        gT0[c] = lam;
        status[c] = st;
        if (nacc_out) nacc_out[c] = s.nacc;
    }
    if (gcell) {
        wave_sync();
#pragma unroll 1
        for (int j = lane; j < R; j += WAVE)
            gcell[(int64_t)m.rx[j].orig * n_cells + c] = ok ? TH[j] : __longlong_as_double(0x7ff8000000000000ll);
    }
    wave_sync();
}

template <int NP>
__global__ void __launch_bounds__(WAVE) k_adjoint(DevMech mk, Opts o, int64_t n, const double *T0, const double *P,
                                                  const double *Y0, int64_t ld, const double *DT,
                                                  const double *dlnA, const double *h_in, const double *gT1,
                                                  const double *gY1, double *gT0, double *gY0, double *gcell,
                                                  int32_t *status, int32_t *nacc, double *T1, double *Y1,
                                                  double *scratch, int64_t slot_doubles, int hcap,
                                                  unsigned long long *queue, const int32_t *perm)
{
    extern __shared__ double lds[];
    const DevMech m = fix_reactor<false>(mk);  // constant pressure only
    const int lane = threadIdx.x;
    double *slot = scratch + (int64_t)blockIdx.x * slot_doubles;
#pragma unroll 1
    while (true) {
        unsigned long long i = 0;
        if (lane == 0) i = atomicAdd(queue, 1ull);
        i = __shfl(i, 0, WAVE);
        if (i >= (unsigned long long)n) break;
        const int64_t c = perm ? (int64_t)perm[i] : (int64_t)i;
        adjoint_cell<NP>(m, o, lds, c, lane, T0, P, Y0, ld, DT, dlnA, h_in, gT1, gY1, gT0, gY0, gcell, n, status,
                         nacc, T1, Y1, slot, hcap);
    }
}

// Vector-Jacobian product of the right-hand side at n states.
template <int NP>
__global__ void __launch_bounds__(WAVE) k_vjp(DevMech mk, int64_t n, const double *T, const double *P,
                                              const double *Y, int64_t ld, const double *dlnA, const double *wT,
                                              const double *wY, double *gT, double *gY, double *gcell)
{
    extern __shared__ double lds[];
    const DevMech m = fix_reactor<false>(mk);  // constant pressure only
    const int lane = threadIdx.x;
    const int64_t c = blockIdx.x;
    if (c >= n) return;
    double *TH = lds + LdsA<NP>::TH;
#pragma unroll 1
    for (int j = lane; j < m.R; j += WAVE) TH[j] = 0.0;
    const double y = load_state(m, T, Y, ld, c, lane);
    const double w = load_state(m, wT, wY, ld, c, lane);
    wave_sync();
    const double g = vjp<NP, double>(m, lds, y, P[c], dlnA, w, lane, TH);
    if (lane < m.N) gY[(int64_t)lane * ld + c] = g;
    if (lane == m.N) gT[c] = g;
    if (gcell) {
#pragma unroll 1
        for (int j = lane; j < m.R; j += WAVE) gcell[(int64_t)m.rx[j].orig * n + c] = TH[j];
    }
}

// out[j] = sum_c g[j*n + c], one block per reaction, in a fixed order (the
// result does not depend on how cells were scheduled).
__global__ void __launch_bounds__(256) k_sum_cells(const double *g, int64_t n, double *out)
{
    __shared__ double part[256];
    const int j = blockIdx.x;
    const int t = threadIdx.x;
    double s = 0.0;
    for (int64_t c = t; c < n; c += 256) s += g[(int64_t)j * n + c];
    part[t] = s;
    __syncthreads();
#pragma unroll
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) part[t] += part[t + w];
        __syncthreads();
    }
    if (t == 0) out[j] = part[0];
}

// ---------------------------------------------------------------------------
// launchers (host)
// ---------------------------------------------------------------------------
template <int NP>
size_t lds_bytes_adj(int R)
{
    return sizeof(double) * ((size_t)LdsA<NP>::fixed() + (size_t)R);
}

#define SC_DISPATCH_A(np, CALL)                       \
    switch (np) {                                     \
    case 16: { constexpr int NPV = 16; CALL; } break; \
    case 32: { constexpr int NPV = 32; CALL; } break; \
    case 56: { constexpr int NPV = 56; CALL; } break; \
    case 64: { constexpr int NPV = 64; CALL; } break; \
    default: return hipErrorInvalidValue;             \
    }

int adjoint_slot_checkpoints() { return NCK; }

hipError_t launch_vjp(int np, const DevMech &m, int64_t n, const double *T, const double *p, const double *Y,
                      int64_t ld, const double *dlnA, const double *wT, const double *wY, double *gT, double *gY,
                      double *gcell, hipStream_t s)
{
    SC_DISPATCH_A(np, hipLaunchKernelGGL(k_vjp<NPV>, dim3((unsigned)n), dim3(WAVE), lds_bytes_adj<NPV>(m.R), s, m,
                                         n, T, p, Y, ld, dlnA, wT, wY, gT, gY, gcell));
    return hipGetLastError();
}

hipError_t launch_adjoint(int np, const DevMech &m, const Opts &o, int64_t n, const double *T0, const double *p,
                          const double *Y0, int64_t ld, const double *dt, const double *dlnA, const double *h_in,
                          const double *gT1, const double *gY1, double *gT0, double *gY0, double *gcell,
                          int32_t *st, int32_t *na, double *T1, double *Y1, double *scratch, int64_t slot_doubles,
                          int hcap, unsigned long long *queue, const int32_t *perm, int grid, hipStream_t s)
{
    SC_DISPATCH_A(np, hipLaunchKernelGGL(k_adjoint<NPV>, dim3((unsigned)grid), dim3(WAVE),
                                         lds_bytes_adj<NPV>(m.R), s, m, o, n, T0, p, Y0, ld, dt, dlnA, h_in, gT1,
                                         gY1, gT0, gY0, gcell, st, na, T1, Y1, scratch, slot_doubles, hcap, queue,
                                         perm));
    return hipGetLastError();
}

hipError_t launch_sum_cells(const double *g, int64_t n, int R, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_cells, dim3((unsigned)R), dim3(256), 0, s, g, n, out);
    return hipGetLastError();
}

int adjoint_capacity(int np, int R, int device)
{
    int per_cu = 0, cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
    hipError_t e = hipErrorInvalidValue;
    switch (np) {
    case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adjoint<16>, WAVE, lds_bytes_adj<16>(R)); break;
    case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adjoint<32>, WAVE, lds_bytes_adj<32>(R)); break;
    case 56: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adjoint<56>, WAVE, lds_bytes_adj<56>(R)); break;
    case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adjoint<64>, WAVE, lds_bytes_adj<64>(R)); break;
    default: break;
    }
    return e == hipSuccess ? per_cu * cus : 0;
}

}  // namespace scdev
