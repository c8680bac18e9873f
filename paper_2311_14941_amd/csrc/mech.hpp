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
constexpr int MAX_STATE = 64;               // N + 1 supported by the one-wave kernels

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
    Counts cnt;
    std::vector<uint8_t> pattern;  // (N+1)^2 structural pattern of the sparse Jacobian terms

    int species(const std::string &s) const;
};

// Parse + validate + compile.  Throws ParseError or Unsupported.
Mech load_mechanism(const std::string &text);

}  // namespace sc
