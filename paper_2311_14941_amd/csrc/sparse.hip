// Kernels with the sparse linear algebra (gfx950): one 64-lane wavefront per
// cell, as in the dense kernels, but the iteration matrix lives in LDS as the
// L+U entries of the bordered system the mechanism compiler built (sparse.cpp)
// and is factorised and solved by following that compiler's static level
// schedules.  State vectors hold VPL components per lane (component
// c = lane + 64 v), so mechanisms of up to 127 species fit one wave.
//
// The bordered system (order N + 2, unknowns z_k = x_k / W_k, x_T, sigma):
//   row k:     z_k/hg - sum_m P_km z_m - us_k sigma - (P_kT/rho + ct us_k) x_T = b_k / W_k
//   row T:     sum_m A_Tm z_m + A_TT x_T = b_T
//   row sigma: vs sum_m z_m - sigma = 0
// with P_km = sum_j nu_kj dq_j/dC_m (the sparse analytical terms, scattered
// reaction by reaction), us_k = UA_k/rho, vs = Wbar, ct = 1/T at constant
// pressure (the density border) and us_k = UA_k, vs = 1, ct = 0 at constant
// volume (the total-concentration border); UA_k = sum_j nu_kj e_j with e_j
// the reaction's Euler remainder (constant pressure) or dq_j/d[M] (constant
// volume).  Eliminating sigma gives back M = I/hg - J exactly (paper
// Sec. 2.5: sparse analytical Jacobian, sparse algebra management).
//
// Every schedule phase is a list of independent items processed 64 at a
// time, four groups in flight; items of one phase that update the same entry
// use LDS atomics, so one wave's results do not depend on anything but the
// schedule (bitwise equal across launch modes).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "core.hpp"

namespace scdev {


// ---------------------------------------------------------------------------
// lane geometry: G lanes per cell.  G = 64: one cell per wave, VPL slots per
// lane.  G = 32 or 16: two or four cells per wave (mechanisms whose N + 2
// positions fit G), each cell in its own aligned group of lanes with one
// slot per lane.  Below, `lane` is the lane within the cell's group; sums
// and broadcasts stay inside the group.
// ---------------------------------------------------------------------------
template <int G>
__device__ __forceinline__ double gsum(double v)
{
#pragma unroll
    for (int off = G / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

template <int G>
__device__ __forceinline__ double gbcast(double v, int k)
{
    if constexpr (G == WAVE)
        return rdlane(v, k);
    else
        return __shfl(v, k, G);
}

template <int G>
__device__ __forceinline__ int gbcast_i(int v, int k)
{
    if constexpr (G == WAVE)
        return __builtin_amdgcn_readlane(v, k);
    else
        return __shfl(v, k, G);
}

template <int G>
__device__ __forceinline__ bool gany(bool b)
{
    if constexpr (G == WAVE)
        return __any(b);
    else
        return gsum<G>(b ? 1.0 : 0.0) > 0.0;
}

// ---------------------------------------------------------------------------
// helpers over VPL components per lane
// ---------------------------------------------------------------------------
template <int VPL, int G = WAVE>
__device__ __forceinline__ double vsum(const double (&a)[VPL])
{
    double s = a[0];
#pragma unroll
    for (int v = 1; v < VPL; ++v) s += a[v];
    return gsum<G>(s);
}

// the temperature component c = N sits in slot N / 64, lane N % 64 (with
// two slots per lane, N = 63 still has it in the first)
template <int VPL, int G = WAVE>
__device__ __forceinline__ double comp_T(const DevMech &m, const double (&y)[VPL])
{
    if (VPL == 1 || m.N < 64) return gbcast<G>(y[0], m.N & 63);
    return gbcast<G>(y[VPL - 1], m.N & 63);
}

template <int VPL, int G = WAVE>
__device__ __forceinline__ void load_state_v(const DevMech &m, const double *T, const double *Y, int64_t ld,
                                             int64_t cell, int lane, double (&y)[VPL])
{
#pragma unroll
    for (int v = 0; v < VPL; ++v) {
        const int c = lane + G * v;
        y[v] = c < m.N ? Y[(int64_t)c * ld + cell] : c == m.N ? T[cell] : 0.0;
    }
}

template <int VPL, int G = WAVE>
__device__ __forceinline__ void store_state_v(const DevMech &m, double *T, double *Y, int64_t ld, int64_t cell,
                                              int lane, const double (&y)[VPL])
{
#pragma unroll
    for (int v = 0; v < VPL; ++v) {
        const int c = lane + G * v;
        if (c < m.N) Y[(int64_t)c * ld + cell] = y[v];
        if (c == m.N) T[cell] = y[v];
    }
}

// ---------------------------------------------------------------------------
// thermodynamics, right-hand side and Jacobian terms
// ---------------------------------------------------------------------------
// Mixture state from y; writes C, g/RT, h/RT and clears the accumulators.
template <int VPL, int G = WAVE>
__device__ __forceinline__ Mix<> mixture_v(const DevMech &m, const DevSparse &sp, double *lds,
                                           const double (&y)[VPL], double p, Thermo<> (&th)[VPL], int lane)
{
    const int N = m.N;
    Mix<> x;
    x.T = comp_T<VPL, G>(m, y);
    x.invT = 1.0 / x.T;
    x.lnT = log(x.T);
    x.p = p;
    double yw[VPL], cpw[VPL];
#pragma unroll
    for (int v = 0; v < VPL; ++v) {
        const int c = lane + G * v;
        th[v] = Thermo<>{0.0, 0.0, 0.0, 0.0};
        yw[v] = cpw[v] = 0.0;
        if (c < N) {
            th[v] = nasa7<double>(m, c, x.T, x.lnT, x.invT);
            yw[v] = y[v] * m.invW()[c];
            cpw[v] = th[v].cpR * yw[v];
        }
    }
    x.Wbar = 1.0 / vsum<VPL, G>(yw);
    x.cp = m.Rgas * vsum<VPL, G>(cpw);
    if (m.cv) {
        x.rho = p;
        x.p = p * m.Rgas * x.T / x.Wbar;
        x.cp = x.cp - m.Rgas / x.Wbar;
    } else {
        x.rho = p * x.Wbar * x.invT / m.Rgas;
    }
#pragma unroll
    for (int v = 0; v < VPL; ++v) {
        const int c = lane + G * v;
        if (c < N) {
            lds[sp.C + c] = x.rho * yw[v];
            lds[sp.G + c] = th[v].hRT - th[v].sR;
            lds[sp.H + c] = th[v].hRT;
            lds[sp.WD + c] = 0.0;
        }
        if (c <= N) lds[sp.UA + c] = 0.0;
    }
    return x;
}

// A kernel instantiated without the tables sees a null table pointer as a
// compile-time constant, so the tables' code paths fold away.
template <bool TB>
__device__ __forceinline__ DevSparse fix_tables(DevSparse sp)
{
    if constexpr (!TB) sp.itab = nullptr;
    return sp;
}

// With interpolated thermodynamics: the cell's interval of the table (its
// reactions' coefficient blocks) and the local coordinate t in [-1, 1];
// null for exact thermodynamics or a T outside the table's range.
__device__ __forceinline__ const double *thermo_block(const DevSparse &sp, int R, double lnT, double &t)
{
    t = 0.0;
    if (!sp.itab) return nullptr;
    const double uu = (lnT - sp.iu0) * sp.iinvdu;
    if (!(uu >= 0.0) || !(uu < (double)sp.inint)) return nullptr;
    const int iv = (int)uu;
    t = 2.0 * (uu - iv) - 1.0;
    return sp.itab + (size_t)iv * R * 2 * (sp.ideg + 1);
}

// f(y): dY_k/dt and dT/dt, VPL components per lane (0 beyond N).
template <int VPL, int G = WAVE>
__device__ __forceinline__ void rhs_v(const DevMech &m, const DevSparse &sp, double *lds, const double (&y)[VPL], double p,
                      const double *dlnA, int lane, double (&f)[VPL])
{
    const int N = m.N, R = m.R;
    Thermo<> th[VPL];
    const Mix<> x = mixture_v<VPL, G>(m, sp, lds, y, p, th, lane);
    double itt;
    const double *itb = thermo_block(sp, R, x.lnT, itt);
    __syncthreads();
    // the reaction loop, compiled once with the tables and once without (the
    // exact path's code does not carry the tables' branches)
    auto pass = [&](auto tables) __attribute__((always_inline)) {
#pragma unroll 1
        for (int j = lane; j < R; j += G) {
            const RxRec rr = load_rec(m, j);
            const double dl = dlnA ? dlnA[rr.orig] : 0.0;
            RxOut<> o;
            if constexpr (decltype(tables)::value)
                o = reaction<false>(m, lds, rr, x, dl, sp.C, sp.G, sp.H, 0, itb + (size_t)j * 2 * (sp.ideg + 1), itt,
                                    sp.ideg);
            else
                o = reaction<false>(m, lds, rr, x, dl, sp.C, sp.G, sp.H);
#pragma unroll
            for (int i = 0; i < sc::MAXSIDE; ++i) {
                if (i < rr.nr) atomicAdd(&lds[sp.WD + rr.rsp[i]], -(double)rr.rnu[i] * o.q);
                if (i < rr.np) atomicAdd(&lds[sp.WD + rr.psp[i]], (double)rr.pnu[i] * o.q);
            }
        }
    };
    if (itb)
        pass(std::true_type{});
    else
        pass(std::false_type{});
    __syncthreads();
    double hw[VPL];
#pragma unroll
    for (int v = 0; v < VPL; ++v) {
        const int c = lane + G * v;
        f[v] = hw[v] = 0.0;
        if (c < N) {
            const double wd = lds[sp.WD + c];
            f[v] = m.W()[c] * wd / x.rho;
            hw[v] = (m.cv ? th[v].hRT - 1.0 : th[v].hRT) * wd;
        }
    }
    const double fT = -m.Rgas * x.T * vsum<VPL, G>(hw) / (x.rho * x.cp);
#pragma unroll
    for (int v = 0; v < VPL; ++v)
        if (lane + G * v == N) f[v] = fT;
    __syncthreads();
}

// Jacobian pass: f(y), and the bordered matrix of I/hg - J formed in the L+U
// entries (fill entries zero).  The reaction loop scatters -nu dq/dC and
// -nu dq/dT into the species rows and the reaction-enthalpy-weighted
// derivatives into the temperature row; the border entries are finished per
// state component after one barrier.
template <int VPL, int G = WAVE>
__device__ __forceinline__ void jac_v(const DevMech &m, const DevSparse &sp, double *lds, const double (&y)[VPL], double p,
                      const double *dlnA, int lane, double inv_hg, double (&f)[VPL])
{
    const int N = m.N, R = m.R;
    double *E = lds + sp.E;
    Thermo<> th[VPL];
    const Mix<> x = mixture_v<VPL, G>(m, sp, lds, y, p, th, lane);
#pragma unroll 4
    for (int e = lane; e <= sp.nnz; e += G) E[e] = 0.0;  // and the zero slot E[nnz]
    __syncthreads();
    const double RT = m.Rgas * x.T;
    double itt;
    const double *itb = thermo_block(sp, R, x.lnT, itt);
    auto pass = [&](auto tables) __attribute__((always_inline)) {
#pragma unroll 1
    for (int j = lane; j < R; j += G) {
        const RxRec rr = load_rec(m, j);
        const double dl = dlnA ? dlnA[rr.orig] : 0.0;
        RxOut<> o;
        if constexpr (decltype(tables)::value)
            o = reaction<true>(m, lds, rr, x, dl, sp.C, sp.G, sp.H, 0, itb + (size_t)j * 2 * (sp.ideg + 1), itt,
                               sp.ideg);
        else
            o = reaction<true>(m, lds, rr, x, dl, sp.C, sp.G, sp.H);
        // the reaction's entry indices are loaded once its rate terms are
        // done, so they do not hold registers through the rate arithmetic
        __builtin_amdgcn_sched_barrier(0);
        uint16_t ix[sc::RXI_SIZE];
        __builtin_memcpy(ix, sp.rxi + (size_t)j * sc::RXI_SIZE, sizeof ix);
        // temperature-row weight: the reaction enthalpy (constant pressure) or
        // internal energy (constant volume), per unit of progress
        const double dHJ = m.cv ? (o.dH - rr.dnu) * RT : o.dH * RT;
        bool use[sc::NDEP];
#pragma unroll
        for (int i = 0; i < sc::MAXSIDE; ++i) {
            use[i] = i < rr.nr;
            use[3 + i] = i < rr.np;
        }
#pragma unroll
        for (int e = 0; e < sc::MAXENH; ++e) use[6 + e] = e < rr.neff;
#pragma unroll
        for (int r = 0; r < 2 * sc::MAXSIDE; ++r) {
            const bool isr = r < sc::MAXSIDE;
            const int ri = isr ? r : r - sc::MAXSIDE;
            if (ri >= (isr ? rr.nr : rr.np)) continue;
            const int row = isr ? rr.rsp[ri] : rr.psp[ri];
            const double nu = isr ? -(double)rr.rnu[ri] : (double)rr.pnu[ri];
            atomicAdd(&lds[sp.WD + row], nu * o.q);
            atomicAdd(&lds[sp.UA + row], nu * o.euler);
#pragma unroll
            for (int s = 0; s < sc::NDEP; ++s)
                if (use[s]) atomicAdd(&E[ix[r * sc::RXI_ROW + s]], -nu * o.d[s]);
            atomicAdd(&E[ix[r * sc::RXI_ROW + sc::NDEP]], -nu * o.dT);
        }
#pragma unroll
        for (int s = 0; s < sc::NDEP; ++s)
            if (use[s]) atomicAdd(&E[ix[sc::RXI_TROW + s]], dHJ * o.d[s]);
        atomicAdd(&E[ix[sc::RXI_TROW + sc::NDEP]], dHJ * o.dT);
        if (m.cv) atomicAdd(&lds[sp.UA + N], dHJ * o.euler);
    }
    };
    if (itb)
        pass(std::true_type{});
    else
        pass(std::false_type{});
    __syncthreads();
    const double one = m.cv ? 1.0 : 0.0;
    double hw[VPL], eu[VPL], cpf[VPL], dcp[VPL];
#pragma unroll
    for (int v = 0; v < VPL; ++v) {
        const int c = lane + G * v;
        f[v] = hw[v] = eu[v] = cpf[v] = dcp[v] = 0.0;
        if (c < N) {
            const double Wk = m.W()[c], iw = m.invW()[c];
            const double wd = lds[sp.WD + c], ua = lds[sp.UA + c];
            f[v] = Wk * wd / x.rho;
            hw[v] = (th[v].hRT - one) * wd;
            eu[v] = th[v].hRT * ua / x.rho;      // (h_k/(R T W_k)) u_k, u_k = W_k UA_k / rho
            cpf[v] = (th[v].cpR - one) * f[v] * iw;
            dcp[v] = th[v].dcpR * y[v] * iw;
        }
    }
    const double H = RT * vsum<VPL, G>(hw);
    const double Eu = m.cv ? 0.0 : RT * vsum<VPL, G>(eu);
    const double Scpf = m.Rgas * vsum<VPL, G>(cpf);
    const double Sdcp = m.Rgas * vsum<VPL, G>(dcp);
    const double fT = -H / (x.rho * x.cp);
    const double vs = m.cv ? 1.0 : x.Wbar;
    const double ct = m.cv ? 0.0 : x.invT;
    const double tb = m.cv ? lds[sp.UA + N] : x.Wbar * Eu;
    const double icp = 1.0 / x.cp;
#pragma unroll
    for (int v = 0; v < VPL; ++v) {
        const int c = lane + G * v;
        if (c < N) {
            const int32_t *cm = sp.comp + CMP * c;
            const double us = m.cv ? lds[sp.UA + c] : lds[sp.UA + c] / x.rho;
            E[cm[1]] += inv_hg;
            E[cm[2]] = E[cm[2]] / x.rho - ct * us;
            E[cm[3]] = -us;
            E[cm[4]] = (E[cm[4]] + tb + fT * m.Rgas * (th[v].cpR - one)) * icp;
            E[cm[5]] = vs;
        } else if (c == N) {
            f[v] = fT;
            const int32_t *cm = sp.comp + CMP * N;
            const double eT = m.cv ? 0.0 : Eu * x.invT;
            E[cm[1]] = inv_hg + (E[cm[1]] / x.rho + eT + Scpf + fT * Sdcp) * icp;
            E[cm[2]] = -1.0;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// schedules
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lo16(uint64_t x) { return (int)(x & 0xffff); }
__device__ __forceinline__ int mid16(uint64_t x) { return (int)((x >> 16) & 0xffff); }
__device__ __forceinline__ int hi16(uint64_t x) { return (int)((x >> 32) & 0xffff); }

// The first four G-item groups of a phase, loaded ahead (the loads of the
// next phase are issued before the current one is processed, so their
// latency overlaps its LDS work).
struct Pre {
    uint64_t it[4];
};
template <int G>
__device__ __forceinline__ Pre preload(const uint64_t *items, int q0, int q1, int lane)
{
    Pre p;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int q = q0 + u * G + lane;
        p.it[u] = q < q1 ? items[q] : ~0ull;
    }
    return p;
}

// l_ik = a_ik / a_kk for the items of one phase (b items: e_ik | e_kk << 16)
__device__ __forceinline__ void lu_scale_items(double *E, const uint64_t (&it)[4])
{
    double a[4], d[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const bool ok = it[u] != ~0ull;
        a[u] = ok ? E[lo16(it[u])] : 0.0;
        d[u] = ok ? E[mid16(it[u])] : 1.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (it[u] != ~0ull) E[lo16(it[u])] = a[u] / d[u];
}

// a_ij -= l_ik u_kj for the items of one phase (c items: e_ij | e_ik << 16 | e_kj << 32)
__device__ __forceinline__ void lu_update_items(double *E, const uint64_t (&it)[4])
{
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const bool ok = it[u] != ~0ull;
        a[u] = ok ? E[mid16(it[u])] : 0.0;
        b[u] = ok ? E[hi16(it[u])] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (it[u] != ~0ull) atomicAdd(&E[lo16(it[u])], -a[u] * b[u]);
}

// The dense trailing block [t0, n) (w = n - t0 <= W positions, full L+U
// pattern) in registers: lane r holds row t0 + r, columns t0..n-1.  The
// rows of the block are the last w entries of each of its columns (entries
// are numbered column by column), so no index table is read.  Right-looking
// elimination: per pivot k, the pivot row is broadcast entry by entry and
// every row below applies it; rows at or above the pivot multiply by zero.
// Padding (rows and columns from w to W) holds zeros and takes part
// unconditionally: the loops have fixed trip counts, the array stays in
// registers.  L is stored scaled (l_ik = a_ik / a_kk), U and the diagonal
// as computed.  The same operations as the level schedule would perform,
// without its barriers and schedule loads (one level per pivot in a dense
// block).
template <int G, int W>
__device__ __forceinline__ void lu_tail(const DevSparse &sp, double *E, int lane)
{
    const int n = sp.n, t0 = sp.tail0, w = n - t0;
    const bool row = lane < w;
    const int back = n - t0 - lane;  // entry (t0 + lane, c) = cstart[c + 1] - back
    const int cend = row ? sp.cstart[t0 + lane + 1] : 0;  // lane j: end of column t0 + j
    double a[W];
    // loads at a clamped index and selects (no lane mask per column is kept
    // alive until the stores)
#pragma unroll
    for (int j = 0; j < W; ++j) {
        const int e = gbcast_i<G>(cend, j) - back;
        const bool ok = j < w && row;
        const double x = E[ok ? e : 0];
        a[j] = ok ? x : 0.0;
    }
#pragma unroll
    for (int k = 0; k < W - 1; ++k) {
        const double akk = gbcast<G>(a[k], k);
        const bool sub = row && lane > k;  // a row below the pivot
        const double l = sub ? a[k] / akk : 0.0;
        a[k] = sub ? l : a[k];
#pragma unroll
        for (int j = k + 1; j < W; ++j) a[j] = fma(-l, gbcast<G>(a[j], k), a[j]);
    }
#pragma unroll
    for (int j = 0; j < W; ++j) {
        const int e = gbcast_i<G>(cend, j) - back;
        if (j < w && row) E[e] = a[j];
    }
}

// Numeric LU of the formed matrix in E: the static level schedule of the
// pivots before the dense tail, the tail in registers, then dinv = 1/u_kk
// and the rows of U scaled to a unit diagonal.
template <int VPL, int G>
__device__ void lu_v(const DevSparse &sp, double *lds, int lane)
{
    double *E = lds + sp.E;
    double *DINV = lds + sp.DINV;
    Pre pre = preload<G>(sp.lu_b, sp.lu_b_lvl[0], sp.lu_b_lvl[1], lane);
#pragma unroll 1
    for (int l = 0; l < sp.nl_lu; ++l) {
        const int b0 = sp.lu_b_lvl[l], b1 = sp.lu_b_lvl[l + 1];
        const int c0 = sp.lu_c_lvl[l], c1 = sp.lu_c_lvl[l + 1];
        Pre cur = pre;
        pre = preload<G>(sp.lu_c, c0, c1, lane);
        lu_scale_items(E, cur.it);
#pragma unroll 1
        for (int base = b0 + 4 * G; base < b1; base += 4 * G)
            lu_scale_items(E, preload<G>(sp.lu_b, base, b1, lane).it);
        __syncthreads();
        cur = pre;
        if (l + 1 < sp.nl_lu) pre = preload<G>(sp.lu_b, b1, sp.lu_b_lvl[l + 2], lane);
        if (c1 > c0) {
            lu_update_items(E, cur.it);
#pragma unroll 1
            for (int base = c0 + 4 * G; base < c1; base += 4 * G)
                lu_update_items(E, preload<G>(sp.lu_c, base, c1, lane).it);
            __syncthreads();
        }
    }
    // the tail width the kernel holds: one slot per lane (n <= 64) or two
    constexpr int W = VPL == 1 ? (G < sc::SPARSE_TAIL_MAX ? G : sc::SPARSE_TAIL_MAX) : sc::SPARSE_TAIL_MAX_WIDE;
    lu_tail<G, W>(sp, E, lane);
    __syncthreads();
#pragma unroll 1
    for (int k = lane; k < sp.n; k += G) DINV[k] = 1.0 / E[sp.diag[k]];
    __syncthreads();
#pragma unroll 2
    for (int q = lane; q < sp.n_u; q += G) {
        const uint32_t it = sp.lu_u[q];
        E[it & 0xffff] *= DINV[it >> 16];
    }
    __syncthreads();
}

// Solve M x = b with the factors in E (b, x: VPL components per lane).
// The vector is moved to position order and swept in registers, one column
// of L (then of the unit-diagonal U) per iteration: the pivot value is
// broadcast with readlane and every lane whose row holds an entry in that
// column updates its component.  Entries are numbered column by column, so
// a lane's entry in column k is the column's start plus the number of
// entries in the rows above it: a count of the column's row mask below the
// lane (mbcnt), with the mask and start read as wave-uniform values.  No
// barrier and no per-lane index load inside the sweeps.
template <int VPL, int G = WAVE>
__device__ __forceinline__ double rd_pos(const double (&z)[VPL], int k)
{
    if (VPL == 1 || k < 64) return gbcast<G>(z[0], k);
    return gbcast<G>(z[VPL - 1], k - 64);
}

// bits of m below this lane's position in its group (mbcnt for a whole wave)
template <int G>
__device__ __forceinline__ int below(uint64_t m, int lane)
{
    if constexpr (G == WAVE)
        return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    else
        return __builtin_popcountll(m & ((1ull << lane) - 1));
}

template <int G>
__device__ __forceinline__ uint64_t gbcast64(uint64_t v, int k)
{
    const uint32_t lo = (uint32_t)gbcast_i<G>((int)(uint32_t)v, k);
    const uint32_t hi = (uint32_t)gbcast_i<G>((int)(uint32_t)(v >> 32), k);
    return (uint64_t)hi << 32 | lo;
}

// The columns' row masks and entry starts, held one column per lane
// (column lane + 64 w in slot w), loaded once per solve.
template <int VPL, int G = WAVE>
struct ColMeta {
    uint64_t m0[VPL], m1[VPL];
    int start[VPL];
};

template <int VPL, int G = WAVE>
__device__ __forceinline__ ColMeta<VPL, G> col_meta(const DevSparse &sp, int lane)
{
    ColMeta<VPL, G> c;
#pragma unroll
    for (int w = 0; w < VPL; ++w) {
        const int k = lane + G * w;
        const bool ok = k < sp.n;
        c.m0[w] = ok ? sp.cmask[2 * k] : 0;
        c.m1[w] = ok && VPL > 1 ? sp.cmask[2 * k + 1] : 0;
        c.start[w] = ok ? sp.cstart[k] : 0;
    }
    return c;
}

// This lane's factor value in column k for each slot (0 where its row has
// no entry there).  An absent entry's index still lies inside the LDS
// allocation (at most the column's end), and the select keeps whatever it
// holds out of the result.
template <int VPL, int G = WAVE>
__device__ __forceinline__ void col_values(const ColMeta<VPL, G> &c, const double *E, int k, int lane,
                                           double (&val)[VPL])
{
    const int w = VPL == 1 ? 0 : k >> 6, kk = k & 63;
    const uint64_t m0 = gbcast64<G>(c.m0[w], kk);
    const int base = gbcast_i<G>(c.start[w], kk);
    val[0] = (m0 >> lane) & 1 ? E[base + below<G>(m0, lane)] : 0.0;
    if (VPL > 1) {
        const uint64_t m1 = gbcast64<G>(c.m1[w], kk);
        val[VPL - 1] = (m1 >> lane) & 1 ? E[base + __builtin_popcountll(m0) + below<G>(m1, lane)] : 0.0;
    }
}

// Column sweeps of a system of at most 64 positions (one slot per lane).
// Lane k of each cell's group holds, for column k, the mask of the rows
// below (forward) and above (backward) the diagonal that hold an entry and
// the first of those entries; a sweep broadcasts them per column
// (readlane, or a group shuffle), and a lane's entry is that start plus the
// mask's bits below the lane.  The LDS read is unconditional (the index
// never leaves the column's entries) and the lanes without an entry are
// zeroed by a select on the mask; the select is applied one column later,
// so the read of column k + 1 overlaps the update with column k.  No
// branch, no barrier.
// v where the lane's bit of the lane mask m is set, else 0 (one
// v_cndmask per half with the mask as the lane condition)
__device__ __forceinline__ double keep_lanes(uint64_t m, double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    int rlo, rhi;
    asm("v_cndmask_b32 %0, 0, %1, %2" : "=v"(rlo) : "v"(lo), "s"(m));
    asm("v_cndmask_b32 %0, 0, %1, %2" : "=v"(rhi) : "v"(hi), "s"(m));
    return __hiloint2double(rhi, rlo);
}

struct SweepCol {
    uint64_t msk;  // rows of the column holding an entry
    double raw;    // the LDS word read for this lane (meaningless off the mask)
};

template <int G>
__device__ __forceinline__ SweepCol sweep_col(int mlo, int mhi, int start, const double *E, int k, int lane)
{
    const uint64_t msk = (uint64_t)(uint32_t)gbcast_i<G>(mhi, k) << 32 | (uint32_t)gbcast_i<G>(mlo, k);
    const int e = gbcast_i<G>(start, k) + below<G>(msk, lane);
    return SweepCol{msk, E[e]};
}

// the column's value for this lane: with one cell per wave the mask is
// wave-uniform and selects lanes directly; with several cells per wave it
// differs per group and is tested per lane
template <int G>
__device__ __forceinline__ double sweep_value(const SweepCol &c, int lane)
{
    if constexpr (G == WAVE)
        return keep_lanes(c.msk, c.raw);
    else
        return (c.msk >> lane) & 1 ? c.raw : 0.0;
}

// With several cells per wave a broadcast is a group shuffle (an LDS-path
// permute) rather than a readlane, and the three per-column broadcasts of
// mask and start cost more than a table: there each lane reads its entry
// in column k from a per-column row table (the zero slot where it has
// none), four columns ahead, and only the pivot value is broadcast.
template <int G>
__device__ __forceinline__ void sweeps_table(const DevSparse &sp, const double *E, const double *DINV, int n,
                                             int lane, double &z)
{
    const int nc = n - 1, zero = sp.nnz;
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
        // forward: columns 0 .. n-2 (rows below); backward: n-1 .. 1 (rows above)
        const uint16_t *ti = (dir == 0 ? sp.swfi : sp.swbi) + lane;
        auto col = [&](int s) { return dir == 0 ? s : nc - s; };
        int q[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) q[d] = d < nc ? (int)ti[64 * col(d)] : zero;
        double v = E[q[0]];
        int s = 0;
#pragma unroll 1
        for (; s + 4 <= nc; s += 4) {
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const int c = s + d;
                const double vn = c + 1 < nc ? E[q[(d + 1) & 3]] : 0.0;
                q[d] = c + 4 < nc ? (int)ti[64 * col(c + 4)] : zero;
                z = fma(-v, gbcast<G>(z, col(c)), z);
                v = vn;
            }
        }
#pragma unroll 1
        for (; s < nc; ++s) {
            const double vn = s + 1 < nc ? E[(int)ti[64 * col(s + 1)]] : 0.0;
            z = fma(-v, gbcast<G>(z, col(s)), z);
            v = vn;
        }
        if (dir == 0 && lane < n) z *= DINV[lane];
    }
}

template <int G>
__device__ __forceinline__ void sweeps_1(const DevSparse &sp, const double *E, const double *DINV, int n, int lane,
                                         double &z)
{
    if constexpr (G < WAVE) {
        sweeps_table<G>(sp, E, DINV, n, lane, z);
        return;
    }
    const bool live = lane < n;
    const uint32_t *f = sp.swf + 4 * (live ? lane : 0), *b = sp.swb + 4 * (live ? lane : 0);
    const int flo = live ? (int)f[0] : 0, fhi = live ? (int)f[1] : 0, fst = live ? (int)f[2] : 0;
    const int blo = live ? (int)b[0] : 0, bhi = live ? (int)b[1] : 0, bst = live ? (int)b[2] : 0;
    // forward with the unit-diagonal L, k ascending
    SweepCol nxt = sweep_col<G>(flo, fhi, fst, E, 0, lane);
    for (int k = 0; k < n - 1; ++k) {
        const SweepCol cur = nxt;
        if (k + 1 < n - 1) nxt = sweep_col<G>(flo, fhi, fst, E, k + 1, lane);
        z = fma(-sweep_value<G>(cur, lane), gbcast<G>(z, k), z);
    }
    if (live) z *= DINV[lane];
    // backward with the unit-diagonal U, k descending
    nxt = sweep_col<G>(blo, bhi, bst, E, n - 1, lane);
    for (int k = n - 1; k > 0; --k) {
        const SweepCol cur = nxt;
        if (k > 1) nxt = sweep_col<G>(blo, bhi, bst, E, k - 1, lane);
        z = fma(-sweep_value<G>(cur, lane), gbcast<G>(z, k), z);
    }
}

template <int VPL, int G = WAVE>
__device__ void solve_v(const DevMech &m, const DevSparse &sp, double *lds, const double (&b)[VPL], int lane,
                        double (&x)[VPL])
{
    const int N = m.N, n = sp.n;
    const double *E = lds + sp.E;
    double *X = lds + sp.X;
    const double *DINV = lds + sp.DINV;
    const ColMeta<VPL, G> cm = col_meta<VPL, G>(sp, lane);
#pragma unroll
    for (int v = 0; v < VPL; ++v) {
        const int c = lane + G * v;
        if (c < N) X[sp.comp[CMP * c]] = b[v] * m.invW()[c];
        if (c == N) X[sp.comp[CMP * N]] = b[v];
    }
    if (lane == 0) X[n - 1] = 0.0;  // sigma row
    __syncthreads();
    double z[VPL];
#pragma unroll
    for (int v = 0; v < VPL; ++v) {
        const int q = lane + G * v;
        z[v] = q < n ? X[q] : 0.0;
    }
    if constexpr (VPL == 1) {
        sweeps_1<G>(sp, E, DINV, n, lane, z[0]);
    } else {
    // forward: x_i -= l_ik x_k, k ascending, rows below the diagonal (the
    // next column's values are read while this one is applied)
    double nxt[VPL], cur[VPL];
    col_values<VPL, G>(cm, E, 0, lane, nxt);
    for (int k = 0; k < n - 1; ++k) {
#pragma unroll
        for (int v = 0; v < VPL; ++v) cur[v] = nxt[v];
        if (k + 1 < n - 1) col_values<VPL, G>(cm, E, k + 1, lane, nxt);
        const double zk = rd_pos<VPL, G>(z, k);
#pragma unroll
        for (int v = 0; v < VPL; ++v)
            if (lane + G * v > k) z[v] = fma(-cur[v], zk, z[v]);
    }
#pragma unroll
    for (int v = 0; v < VPL; ++v) {
        const int q = lane + G * v;
        if (q < n) z[v] *= DINV[q];
    }
    // backward with the unit-diagonal U: x_i -= u'_ik x_k, k descending,
    // rows above the diagonal
    col_values<VPL, G>(cm, E, n - 1, lane, nxt);
    for (int k = n - 1; k > 0; --k) {
#pragma unroll
        for (int v = 0; v < VPL; ++v) cur[v] = nxt[v];
        if (k > 1) col_values<VPL, G>(cm, E, k - 1, lane, nxt);
        const double zk = rd_pos<VPL, G>(z, k);
#pragma unroll
        for (int v = 0; v < VPL; ++v)
            if (lane + G * v < k) z[v] = fma(-cur[v], zk, z[v]);
    }
    }
    __syncthreads();  // every lane has read X
#pragma unroll
    for (int v = 0; v < VPL; ++v) {
        const int q = lane + G * v;
        if (q < n) X[q] = z[v];
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < VPL; ++v) {
        const int c = lane + G * v;
        x[v] = c < N ? X[sp.comp[CMP * c]] * m.W()[c] : c == N ? X[sp.comp[CMP * N]] : 0.0;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// one Rosenbrock attempt and the integration of a cell
// ---------------------------------------------------------------------------
template <int VPL, int G = WAVE>
__device__ void ros_attempt_v(const DevMech &m, const DevSparse &sp, const Opts &o, double *lds,
                              const double (&y)[VPL], double p, const double *dlnA, int lane, double hc, double *err,
                              double (&ynew)[VPL])
{
    const int n = m.N + 1;
    double *U = lds + sp.U;
    const int NV = sp.NV;
    double f0[VPL], flast[VPL];
    jac_v<VPL, G>(m, sp, lds, y, p, dlnA, lane, 1.0 / (GAM * hc), f0);
    lu_v<VPL, G>(sp, lds, lane);
    const double ih = 1.0 / hc;
#pragma unroll
    for (int v = 0; v < VPL; ++v) flast[v] = f0[v];
#pragma unroll 1
    for (int i = 0; i < NS; ++i) {
        double fi[VPL];
        const int reuse = TREUSE[i];
        if (reuse == 0) {
#pragma unroll
            for (int v = 0; v < VPL; ++v) fi[v] = f0[v];
        } else if (reuse > 0) {
#pragma unroll
            for (int v = 0; v < VPL; ++v) fi[v] = flast[v];
        } else {
            double ys[VPL];
#pragma unroll
            for (int v = 0; v < VPL; ++v) {
                ys[v] = y[v];
                for (int j = 0; j < i; ++j) ys[v] += TA[i][j] * U[j * NV + lane + G * v];
            }
            rhs_v<VPL, G>(m, sp, lds, ys, p, dlnA, lane, fi);
#pragma unroll
            for (int v = 0; v < VPL; ++v) flast[v] = fi[v];
        }
        double ui[VPL];
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
            for (int j = 0; j < i; ++j) fi[v] += (TC[i][j] * ih) * U[j * NV + lane + G * v];
            if (lane + G * v >= n) fi[v] = 0.0;
        }
        solve_v<VPL, G>(m, sp, lds, fi, lane, ui);
#pragma unroll
        for (int v = 0; v < VPL; ++v) U[i * NV + lane + G * v] = ui[v];
    }
    double e2[VPL];
#pragma unroll
    for (int v = 0; v < VPL; ++v) {
        double yn = y[v], ev = 0.0;
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            const double ui = U[i * NV + lane + G * v];
            yn += TM[i] * ui;
            ev += TE[i] * ui;
        }
        ynew[v] = yn;
        e2[v] = 0.0;
        if (lane + G * v < n) {
            const double sc = o.atol + o.rtol * fmax(fabs(y[v]), fabs(yn));
            const double r = ev / sc;
            e2[v] = r * r;
        }
    }
    *err = sqrt(vsum<VPL, G>(e2) / n);
}

template <int VPL, int G = WAVE>
__device__ int advance_v(const DevMech &m, const DevSparse &sp, const Opts &o, double *lds, double (&y)[VPL],
                         double p, double dt, const double *dlnA, int lane, Ctl &s)
{
#pragma unroll 1
    while (true) {
        double hc;
        bool last;
        const int st = ctl_begin(s, o, dt, hc, last);
        if (st != SC_CELL_OK) return st;
        double err, ynew[VPL];
        ros_attempt_v<VPL, G>(m, sp, o, lds, y, p, dlnA, lane, hc, &err, ynew);
        const int r = ctl_end(s, o, err, hc, last, dt);
        if (r < 0) return -r;
        if (r == 1) {
#pragma unroll
            for (int v = 0; v < VPL; ++v) y[v] = ynew[v];
            if (last) return SC_CELL_OK;
        }
    }
}

template <int VPL, int G = WAVE>
__device__ __forceinline__ bool bad_input_v(const DevMech &m, const double (&y)[VPL], double p, double dt, int lane)
{
    bool bad = false;
#pragma unroll
    for (int v = 0; v < VPL; ++v) bad = bad || (lane + G * v <= m.N && !isfinite(y[v]));
    const double T = comp_T<VPL, G>(m, y);
    return gany<G>(bad) || !(T > 0.0) || !isfinite(T) || !(p > 0.0) || !isfinite(p) || !(dt >= 0.0) ||
           !isfinite(dt);
}

template <int VPL, int G = WAVE>
__device__ __forceinline__ void integrate_cell_v(const DevMech &m, const DevSparse &sp, const Opts &o, double *lds, int64_t c,
                                 int lane, const double *T0, const double *P, const double *Y0, int64_t ld,
                                 const double *DT, const double *dlnA, double *h_io, double *T1, double *Y1,
                                 int32_t *status, int32_t *nacc_out, int32_t *nrej_out, const int32_t *ref)
{
    // a cell mapped onto another cell's result is left to the mapping pass
    if (ref && ref[c] != c) return;
    double y[VPL];
    load_state_v<VPL, G>(m, T0, Y0, ld, c, lane, y);
    const double p = P[c], dt = DT[c];
    int st = SC_CELL_OK;
    Ctl s = ctl_init(initial_step(h_io, c, dt), dt);
    if (bad_input_v<VPL, G>(m, y, p, dt, lane)) {
        st = SC_CELL_BAD_INPUT;
    } else if (dt > 0.0) {
        st = advance_v<VPL, G>(m, sp, o, lds, y, p, dt, dlnA, lane, s);
    }
    store_state_v<VPL, G>(m, T1, Y1, ld, c, lane, y);
    if (lane == 0) {
        status[c] = st;
        if (nacc_out) nacc_out[c] = s.nacc;
        if (nrej_out) nrej_out[c] = s.nrej;
        if (h_io && st == SC_CELL_OK && dt > 0.0) h_io[c] = s.hnext;
    }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
// One-wave mechanisms (VPL = 1) run two waves per SIMD: their LDS allows it
// (under 20 KB per cell up to 53 species) and the second wave hides the
// first's LDS, memory and broadcast latencies.  The register cap this
// implies spills about a hundred registers to scratch, outside the inner
// loops; measured on the 53-species batch it is still 1.6x faster than one
// wave per SIMD.
#define SP_OCC __attribute__((amdgpu_waves_per_eu(VPL == 1 ? 2 : 1, VPL == 1 ? 2 : 1)))
// CPW cells per wave: each cell takes G = 64 / CPW lanes and its own LDS
// region (sp.size doubles); lane = threadIdx.x % G, group = threadIdx.x / G.
#define SP_GEOMETRY                                   \
    constexpr int G = WAVE / CPW;                     \
    const int lane = (int)threadIdx.x % G;            \
    const int grp = (int)threadIdx.x / G;             \
    double *ldsg = lds + (size_t)grp * sp.size;

template <int VPL, bool CV, int CPW, bool TB>
__global__ void __launch_bounds__(WAVE) SP_OCC k_integrate_sp(DevMech mk, DevSparse spk, Opts o, int64_t n,
                                                       const double *T0, const double *P, const double *Y0,
                                                       int64_t ld, const double *DT, const double *dlnA,
                                                       double *h_io, double *T1, double *Y1, int32_t *status,
                                                       int32_t *nacc, int32_t *nrej, const int32_t *ref)
{
    extern __shared__ double lds[];
    const DevMech m = fix_reactor<CV>(mk);
    const DevSparse sp = fix_tables<TB>(spk);
    SP_GEOMETRY
    const int64_t c = (int64_t)blockIdx.x * CPW + grp;
    if (c >= n) return;
    integrate_cell_v<VPL, G>(m, sp, o, ldsg, c, lane, T0, P, Y0, ld, DT, dlnA, h_io, T1, Y1, status, nacc, nrej,
                             ref);
}

// Each pull takes tile * CPW queue positions; the wave's groups take them
// CPW at a time (a group whose position is past the end idles).
template <int VPL, bool CV, int CPW, bool TB>
__global__ void __launch_bounds__(WAVE) SP_OCC k_integrate_sp_persistent(DevMech mk, DevSparse spk, Opts o, int64_t n,
                                                                  const double *T0, const double *P,
                                                                  const double *Y0, int64_t ld, const double *DT,
                                                                  const double *dlnA, double *h_io, double *T1,
                                                                  double *Y1, int32_t *status, int32_t *nacc,
                                                                  int32_t *nrej, unsigned long long *queue,
                                                                  const int32_t *perm, int tile, const int32_t *ref)
{
    extern __shared__ double lds[];
    const DevMech m = fix_reactor<CV>(mk);
    const DevSparse sp = fix_tables<TB>(spk);
    SP_GEOMETRY
#pragma unroll 1
    while (true) {
        unsigned long long base = 0;
        if (threadIdx.x == 0) base = atomicAdd(queue, (unsigned long long)tile * CPW);
        base = __shfl(base, 0, WAVE);
        if (base >= (unsigned long long)n) break;
        const int64_t end = min((int64_t)base + (int64_t)tile * CPW, n);
#pragma unroll 1
        for (int64_t i = (int64_t)base; i < end; i += CPW) {
            const int64_t q = i + grp;
            if (q < end) {
                const int64_t c = perm ? (int64_t)perm[q] : q;
                integrate_cell_v<VPL, G>(m, sp, o, ldsg, c, lane, T0, P, Y0, ld, DT, dlnA, h_io, T1, Y1, status,
                                         nacc, nrej, ref);
            }
        }
    }
}

template <int VPL, bool CV, int CPW, bool TB>
__global__ void __launch_bounds__(WAVE) SP_OCC k_integrate_sp_static(DevMech mk, DevSparse spk, Opts o, int64_t n,
                                                              const double *T0, const double *P, const double *Y0,
                                                              int64_t ld, const double *DT, const double *dlnA,
                                                              double *h_io, double *T1, double *Y1,
                                                              int32_t *status, int32_t *nacc, int32_t *nrej,
                                                              int64_t group, const int32_t *ref)
{
    extern __shared__ double lds[];
    const DevMech m = fix_reactor<CV>(mk);
    const DevSparse sp = fix_tables<TB>(spk);
    SP_GEOMETRY
    const int64_t c0 = (int64_t)blockIdx.x * group;
    const int64_t c1 = min(c0 + group, n);
#pragma unroll 1
    for (int64_t c = c0 + grp; c < c1; c += CPW)
        integrate_cell_v<VPL, G>(m, sp, o, ldsg, c, lane, T0, P, Y0, ld, DT, dlnA, h_io, T1, Y1, status, nacc,
                                 nrej, ref);
}

template <int VPL, bool CV, int CPW, bool TB>
__global__ void __launch_bounds__(WAVE) k_rhs_sp(DevMech mk, DevSparse spk, int64_t n, const double *T,
                                                 const double *P, const double *Y, int64_t ld, const double *dlnA,
                                                 double *fT, double *fY)
{
    extern __shared__ double lds[];
    const DevMech m = fix_reactor<CV>(mk);
    const DevSparse sp = fix_tables<TB>(spk);
    SP_GEOMETRY
    const int64_t c = (int64_t)blockIdx.x * CPW + grp;
    if (c >= n) return;
    double y[VPL], f[VPL];
    load_state_v<VPL, G>(m, T, Y, ld, c, lane, y);
    rhs_v<VPL, G>(m, sp, ldsg, y, P[c], dlnA, lane, f);
    store_state_v<VPL, G>(m, fT, fY, ld, c, lane, f);
}

// The Jacobian J (dense output, [c][i][j] over (Y, T)) recovered from the
// bordered matrix formed with 1/hg = 0 (the -J of the scaled system with the
// sigma border): eliminating sigma, M'_ij = A_ij + A_i,sigma A_sigma,j, and
// undoing the scaling, J_ij = -(W_i / W_j) M'_ij (species i, j), J_iT =
// -W_i A_iT, J_Tj = -A_Tj / W_j, J_TT = -A_TT.
template <int VPL, bool CV, int CPW, bool TB>
__global__ void __launch_bounds__(WAVE) k_jac_sp(DevMech mk, DevSparse spk, int64_t n, const double *T,
                                                 const double *P, const double *Y, int64_t ld, const double *dlnA,
                                                 double *J)
{
    extern __shared__ double lds[];
    const DevMech m = fix_reactor<CV>(mk);
    const DevSparse sp = fix_tables<TB>(spk);
    SP_GEOMETRY
    const int64_t c = (int64_t)blockIdx.x * CPW + grp;
    if (c >= n) return;
    double y[VPL], f[VPL];
    load_state_v<VPL, G>(m, T, Y, ld, c, lane, y);
    jac_v<VPL, G>(m, sp, ldsg, y, P[c], dlnA, lane, 0.0, f);
    const double *E = ldsg + sp.E;
    const int N = m.N, nn = N + 1, ns = sp.n;
    const int pS = ns - 1;
    auto A = [&](int pi, int pj) {
        const uint16_t e = sp.emap[pi * ns + pj];
        return e == sc::NOENT ? 0.0 : E[e];
    };
#pragma unroll 1
    for (int q = lane; q < nn * nn; q += G) {
        const int i = q / nn, j = q % nn;
        const int pi = sp.comp[CMP * i], pj = sp.comp[CMP * j];  // comp[CMP * N] is pos_T
        double val;
        if (i < N && j < N) val = -(m.W()[i] * m.invW()[j]) * (A(pi, pj) + A(pi, pS) * A(pS, pj));
        else if (i < N) val = -m.W()[i] * A(pi, pj);
        else if (j < N) val = -A(pi, pj) * m.invW()[j];
        else val = -A(pi, pj);
        J[(c * nn + i) * nn + j] = val;
    }
}

template <int VPL, bool CV, int CPW, bool TB>
__global__ void __launch_bounds__(WAVE) k_linsolve_sp(DevMech mk, DevSparse spk, int64_t n, const double *T,
                                                      const double *P, const double *Y, int64_t ld,
                                                      const double *dlnA, const double *hg, const double *b,
                                                      double *x)
{
    extern __shared__ double lds[];
    const DevMech m = fix_reactor<CV>(mk);
    const DevSparse sp = fix_tables<TB>(spk);
    SP_GEOMETRY
    const int64_t c = (int64_t)blockIdx.x * CPW + grp;
    if (c >= n) return;
    double y[VPL], f[VPL], bb[VPL], xx[VPL];
    load_state_v<VPL, G>(m, T, Y, ld, c, lane, y);
    jac_v<VPL, G>(m, sp, ldsg, y, P[c], dlnA, lane, 1.0 / hg[c], f);
    lu_v<VPL, G>(sp, ldsg, lane);
    const int nn = m.N + 1;
#pragma unroll
    for (int v = 0; v < VPL; ++v) {
        const int i = lane + G * v;
        bb[v] = i < nn ? b[c * nn + i] : 0.0;
    }
    solve_v<VPL, G>(m, sp, ldsg, bb, lane, xx);
#pragma unroll
    for (int v = 0; v < VPL; ++v) {
        const int i = lane + G * v;
        if (i < nn) x[c * nn + i] = xx[v];
    }
}

// ---------------------------------------------------------------------------
// launchers (host)
// ---------------------------------------------------------------------------
#define SP_KERNEL(k) k<VPLV, CVV, CPWV, TBV>
#define SP_CASE(vplv, cpwv, ...)                                                                 \
    if (vpl == (vplv) && cpw == (cpwv)) {                                                        \
        constexpr int VPLV = vplv, CPWV = cpwv;                                                  \
        if (m.cv && sp.itab) { constexpr bool CVV = true, TBV = true; __VA_ARGS__; }            \
        else if (m.cv) { constexpr bool CVV = true, TBV = false; __VA_ARGS__; }                 \
        else if (sp.itab) { constexpr bool CVV = false, TBV = true; __VA_ARGS__; }              \
        else { constexpr bool CVV = false, TBV = false; __VA_ARGS__; }                          \
        return hipGetLastError();                                                                \
    }
#define SP_DISPATCH(...)                   \
    SP_CASE(1, 1, __VA_ARGS__)             \
    SP_CASE(1, 2, __VA_ARGS__)             \
    SP_CASE(1, 4, __VA_ARGS__)             \
    SP_CASE(2, 1, __VA_ARGS__)             \
    return hipErrorInvalidValue;

// LDS of one workgroup: one region of sp.size doubles per cell of the wave
static size_t sp_lds(const DevSparse &sp, int cpw) { return sizeof(double) * (size_t)sp.size * cpw; }
static unsigned sp_blocks(int64_t n, int cpw) { return (unsigned)((n + cpw - 1) / cpw); }

hipError_t launch_rhs_sp(int vpl, const DevMech &m, const DevSparse &sp, int64_t n, const double *T,
                         const double *p, const double *Y, int64_t ld, const double *dlnA, double *fT, double *fY,
                         hipStream_t s)
{
    const int cpw = sp.cpw;
    SP_DISPATCH(hipLaunchKernelGGL(SP_KERNEL(k_rhs_sp), dim3(sp_blocks(n, cpw)), dim3(WAVE), sp_lds(sp, cpw), s, m,
                                   sp, n, T, p, Y, ld, dlnA, fT, fY))
}

hipError_t launch_jac_sp(int vpl, const DevMech &m, const DevSparse &sp, int64_t n, const double *T,
                         const double *p, const double *Y, int64_t ld, const double *dlnA, double *J, hipStream_t s)
{
    const int cpw = sp.cpw;
    SP_DISPATCH(hipLaunchKernelGGL(SP_KERNEL(k_jac_sp), dim3(sp_blocks(n, cpw)), dim3(WAVE), sp_lds(sp, cpw), s, m,
                                   sp, n, T, p, Y, ld, dlnA, J))
}

hipError_t launch_linsolve_sp(int vpl, const DevMech &m, const DevSparse &sp, int64_t n, const double *T,
                              const double *p, const double *Y, int64_t ld, const double *dlnA, const double *hg,
                              const double *b, double *x, hipStream_t s)
{
    const int cpw = sp.cpw;
    SP_DISPATCH(hipLaunchKernelGGL(SP_KERNEL(k_linsolve_sp), dim3(sp_blocks(n, cpw)), dim3(WAVE), sp_lds(sp, cpw),
                                   s, m, sp, n, T, p, Y, ld, dlnA, hg, b, x))
}

hipError_t launch_integrate_sp(int vpl, const DevMech &m, const DevSparse &sp, const Opts &o, int64_t n,
                               const double *T0, const double *p, const double *Y0, int64_t ld, const double *dt,
                               const double *dlnA, double *h_io, double *T1, double *Y1, int32_t *st, int32_t *na,
                               int32_t *nr, const int32_t *ref, hipStream_t s)
{
    const int cpw = sp.cpw;
    SP_DISPATCH(hipLaunchKernelGGL(SP_KERNEL(k_integrate_sp), dim3(sp_blocks(n, cpw)), dim3(WAVE), sp_lds(sp, cpw),
                                   s, m, sp, o, n, T0, p, Y0, ld, dt, dlnA, h_io, T1, Y1, st, na, nr, ref))
}

hipError_t launch_integrate_sp_persistent(int vpl, const DevMech &m, const DevSparse &sp, const Opts &o,
                                          int64_t n, const double *T0, const double *p, const double *Y0,
                                          int64_t ld, const double *dt, const double *dlnA, double *h_io,
                                          double *T1, double *Y1, int32_t *st, int32_t *na, int32_t *nr,
                                          unsigned long long *queue, const int32_t *perm, int tile, int grid,
                                          const int32_t *ref, hipStream_t s)
{
    const int cpw = sp.cpw;
    SP_DISPATCH(hipLaunchKernelGGL(SP_KERNEL(k_integrate_sp_persistent), dim3((unsigned)grid), dim3(WAVE),
                                   sp_lds(sp, cpw), s, m, sp, o, n, T0, p, Y0, ld, dt, dlnA, h_io, T1, Y1, st, na,
                                   nr, queue, perm, tile, ref))
}

hipError_t launch_integrate_sp_static(int vpl, const DevMech &m, const DevSparse &sp, const Opts &o, int64_t n,
                                      const double *T0, const double *p, const double *Y0, int64_t ld,
                                      const double *dt, const double *dlnA, double *h_io, double *T1, double *Y1,
                                      int32_t *st, int32_t *na, int32_t *nr, int grid, const int32_t *ref,
                                      hipStream_t s)
{
    const int cpw = sp.cpw;
    const int64_t group = (n + grid - 1) / grid;
    const unsigned g = (unsigned)((n + group - 1) / group);
    SP_DISPATCH(hipLaunchKernelGGL(SP_KERNEL(k_integrate_sp_static), dim3(g), dim3(WAVE), sp_lds(sp, cpw), s, m,
                                   sp, o, n, T0, p, Y0, ld, dt, dlnA, h_io, T1, Y1, st, na, nr, group, ref))
}

int persistent_capacity_sp(int vpl, const DevSparse &sp, int device)
{
    int per_cu = 0, cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
    hipError_t e = hipErrorInvalidValue;
    const int cpw = sp.cpw;
    auto occ = [&](auto kern) { return hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, WAVE, sp_lds(sp, cpw)); };
    if (vpl == 1 && cpw == 1) e = occ(k_integrate_sp_persistent<1, false, 1, false>);
    else if (vpl == 1 && cpw == 2) e = occ(k_integrate_sp_persistent<1, false, 2, false>);
    else if (vpl == 1 && cpw == 4) e = occ(k_integrate_sp_persistent<1, false, 4, false>);
    else if (vpl == 2 && cpw == 1) e = occ(k_integrate_sp_persistent<2, false, 1, false>);
    return e == hipSuccess ? per_cu * cus : 0;
}

}  // namespace scdev
