// Host-side mechanism model and compiler.
//
// The paper's chemistry library keeps "internal sparse algebra management of
// mechanism-related quantities" and a sparse analytical Jacobian (Sec. 2.5).
// Here that is a compile step run once per mechanism: parse and validate the
// text, convert the rate parameters to SI and log form, lay the reactions out
// as structure-of-arrays tables with fixed per-reaction slots (reactant,
// product and enhanced third-body species), derive the sparsity pattern of the
// analytical Jacobian terms, and count the work of every kernel phase.
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace sc {

constexpr int MAXSIDE = 3;                  // distinct species per reaction side
constexpr int MAXENH = 4;                   // enhanced third-body species per reaction
constexpr int NDEP = 2 * MAXSIDE + MAXENH;  // dependency slots per reaction
constexpr int MAX_STATE = 64;               // N + 1 supported by the dense one-wave kernels
constexpr int MAX_STATE_SPARSE = 128;       // N + 1 supported by the sparse kernels (two components per lane)
// widest dense trailing block of the sparse LU held in registers: systems
// of up to 64 positions (two waves per SIMD, a tighter register budget),
// and wider ones (one wave per SIMD)
constexpr int SPARSE_TAIL_MAX = 32;
constexpr int SPARSE_TAIL_MAX_WIDE = 64;
constexpr int sparse_tail_max(int n) { return n <= 64 ? SPARSE_TAIL_MAX : SPARSE_TAIL_MAX_WIDE; }
// per-reaction entry indices of the sparse kernels: for each row slot (3
// reactants, 3 products) the entries of its dependency slots and of the
// temperature column, then the temperature row's entries of the dependency
// slots (unused slots hold NOENT)
constexpr int RXI_ROW = NDEP + 1;
constexpr int RXI_TROW = 2 * MAXSIDE * RXI_ROW;
constexpr int RXI_SIZE = RXI_TROW + NDEP + 2;  // 80 (a 160-byte record)
constexpr uint16_t NOENT = 0xffff;

// The sparse linear algebra of one mechanism (paper Sec. 2.5: the sparse
// analytical Jacobian and the sparse algebra management of the mechanism).
// The iteration matrix M = I/(h gamma) - J is solved through a bordered
// system of order n = N + 2 in the scaled unknowns z_k = x_k / W_k, x_T and
// sigma = (sum_m v_m x_m), in which the species block holds only the terms
// P_km = sum_j nu_kj dq_j/dC_m (fixed sparsity from the reaction list, with
// the third-body concentration rewritten so only enhanced species appear),
// and the dense couplings are two border rows and columns (temperature and
// the density term of constant pressure, or the total concentration of
// constant volume).  The species block is put in minimum-degree order, the
// borders last, so no fill enters the species block from them.  The
// symbolic LU (right-looking, no pivoting) fixes the L+U pattern; the
// numeric work is a static schedule in levels of independent operations.
struct SparseLU {
    int n = 0, nnz = 0;
    std::vector<int> perm;        // position -> variable (species 0..N-1, N = T, N + 1 = sigma)
    std::vector<int> pos;         // variable -> position
    std::vector<int> erow, ecol;  // entry -> (row position, column position), column-major order
    std::vector<int> emap;        // n * n: (row position, column position) -> entry or -1
    std::vector<int> cstart;      // n + 1: first entry of each column
    std::vector<uint64_t> cmask;  // 2 n: rows holding an entry in column j (bits 0-63, 64-127)
    // per column k of a system of at most 64 positions, 4 words each: the
    // rows below the diagonal holding an entry (mask low, high word) and the
    // first of those entries (forward sweep); the same for the rows above
    // the diagonal (backward sweep)
    std::vector<uint32_t> sweep_f, sweep_b;
    // n <= 64: per column k and row i (64 rows per column), the entry of
    // (i, k) below (sweep_fi) or above (sweep_bi) the diagonal, else nnz (a
    // slot the kernels keep at zero)
    std::vector<uint16_t> sweep_fi, sweep_bi;
    std::vector<uint8_t> apat;    // n * n: structural pattern of the bordered matrix (before fill)
    // LU, level by level: scale the L entries of the level's pivots
    // (b items: e_ik | e_kk << 16), then the Schur updates (c items:
    // e_ij | e_ik << 16 | e_kj << 32) whose targets may repeat within a level
    std::vector<int> lu_b_lvl, lu_c_lvl;  // level offsets into b / c items (size levels + 1)
    std::vector<uint32_t> lu_b;
    std::vector<uint64_t> lu_c;
    std::vector<uint32_t> lu_u;           // strict U entries with their pivot: e_kj | k << 16 (row scaling)
    // the dense trailing block [tail0, n) (full L+U pattern, at most
    // sparse_tail_max(n) positions): its pivots are not in the level schedule
    // but factorised in registers after it
    int tail0 = 0;
    std::vector<uint32_t> diag;           // diagonal entry of each position
    // triangular solves (unit L, then the row-scaled unit U): items
    // i | p << 16 | e << 32 meaning x_i -= value(e) x_p, level by level
    std::vector<int> fw_lvl, bw_lvl;
    std::vector<uint64_t> fw, bw;
    // transposed solves (U'^T, then L^T) for the adjoint
    std::vector<int> tfw_lvl, tbw_lvl;
    std::vector<uint64_t> tfw, tbw;
    std::vector<uint16_t> rxi;            // [R][RXI_SIZE] entry indices per reaction, original order
    // entries each state component writes when the matrix is formed: per
    // species k: diagonal, T column, sigma column, T row, sigma row; for T:
    // (T,T), (sigma,sigma), (T,sigma), (sigma,T) (the last two may be absent)
    std::vector<int> e_kk, e_kT, e_kS, e_Tk, e_Sk;
    int e_TT = -1, e_SS = -1, e_TS = -1, e_ST = -1;
    int64_t nnz_a = 0, updates = 0;       // bordered matrix before fill; Schur updates
    int64_t flops_lu = 0, flops_solve = 0;
};

enum RxKind { RX_PLAIN = 0, RX_THIRD = 1, RX_TROE = 2 };

struct ParseError : std::runtime_error {
    using std::runtime_error::runtime_error;
};
struct Unsupported : std::runtime_error {
    using std::runtime_error::runtime_error;
};

struct Reaction {
    int kind = RX_PLAIN;
    double log10A = 0, b = 0, Ea = 0;  // cgs log10 A, J/mol
    std::vector<std::pair<int, int>> reac, prod;
    std::vector<std::pair<int, double>> eff;  // (species, efficiency)
    double troe[7] = {0, 0, 0, 0, 0, 0, 0};  // log10 A0, b0, Ea0, a, T3, T1, T2
};

// Device tables in host memory, structure-of-arrays, reaction index fastest.
struct Tables {
    int N = 0, R = 0, n_troe = 0;
    double Rgas = 0, p0 = 0;
    std::vector<double> W, invW, nasa;  // nasa[c*N + k]
    std::vector<int32_t> kind, nr, np, dnu, neff, tix;
    std::vector<int32_t> rsp, rnu, psp, pnu;  // [slot*R + j]
    std::vector<int32_t> esp;                 // [slot*R + j]
    std::vector<double> eam1;                 // alpha - 1, [slot*R + j]
    std::vector<double> lnA, b, EaR;          // SI, log form
    std::vector<double> troe;                 // [field*n_troe + t]: lnA0, b0, Ea0R, a, 1/T3, 1/T1, T2
};

struct Counts {
    int nnz_jac = 0, nnz_lu = 0;
    int exp_per_rhs = 0;
    int64_t flops_rhs = 0, flops_jac = 0, flops_lu = 0, flops_solve = 0, flops_step = 0;
    int64_t flops_attempt = 0, flops_accept = 0;
    int64_t flops_jac_terms = 0;  // the Jacobian pass beyond its right-hand side (reaction derivative terms)
};

struct Mech {
    std::string name;
    int N = 0, R = 0, E = 0;
    double Rgas = 8.314462618, p0 = 101325.0;
    std::vector<std::string> names, elements;
    std::vector<double> W;
    std::vector<int> comp;    // [k*E + e]
    std::vector<double> nasa; // [k*7 + i]
    std::vector<Reaction> rx;
    int n_third = 0, n_troe = 0;
    int n_padded = 0;
    Tables tab;
    Counts cnt;         // the dense kernels' work
    Counts cnt_sparse;  // the sparse kernels' work (LU and solves from the schedule)
    std::vector<uint8_t> pattern;  // N^2 structural pattern of the species terms P_km (with the diagonal)
    SparseLU sp;

    int species(const std::string &s) const;
};

// Parse + validate + compile.  Throws ParseError or Unsupported.
Mech load_mechanism(const std::string &text);

// Interpolation tables of each reaction's -dG/RT and dH/RT in u = ln T
// (thermo_fit.cpp): per interval, reaction and function the d + 1
// coefficients of the polynomial in t in [-1, 1].
constexpr int THERMO_FIT_MAX_DEGREE = 8;
constexpr int THERMO_FIT_MAX_INTERVALS = 4096;
constexpr size_t THERMO_FIT_TABLE_BYTES = 4u << 20;  // the optimal degree's table limit
struct ThermoFit {
    int degree = 0, nint = 0;
    double Tmin = 0, Tmax = 0, u0 = 0, du = 0, max_err = 0;
    std::vector<double> coef;  // [interval][reaction (mechanism order)][2][degree + 1]
};
// degree 0: the lowest degree whose table meets tol within THERMO_FIT_TABLE_BYTES
ThermoFit fit_thermo(const Mech &m, double Tmin, double Tmax, double tol, int degree);

// The sparse compile (sparse.cpp): ordering, symbolic LU, schedules, entry
// indices and counts of a parsed, validated mechanism.
void compile_sparse(Mech &m);

}  // namespace sc
