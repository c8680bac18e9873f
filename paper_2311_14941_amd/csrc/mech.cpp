// Mechanism text reader, validator and compiler (host side).
#include "mech.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <sstream>

namespace sc {

int Mech::species(const std::string &s) const
{
    for (int k = 0; k < N; ++k)
        if (names[k] == s) return k;
    return -1;
}

namespace {

double to_double(const std::string &t, int line)
{
    char *end = nullptr;
    double v = std::strtod(t.c_str(), &end);
    if (end == t.c_str() || *end != 0 || !std::isfinite(v))
        throw ParseError("line " + std::to_string(line) + ": bad number '" + t + "'");
    return v;
}

int to_int(const std::string &t, int line)
{
    char *end = nullptr;
    long v = std::strtol(t.c_str(), &end, 10);
    if (end == t.c_str() || *end != 0)
        throw ParseError("line " + std::to_string(line) + ": bad integer '" + t + "'");
    return (int)v;
}

// merge repeated species on one side into a single (species, nu) entry
std::vector<std::pair<int, int>> merge_side(const std::vector<std::pair<int, int>> &in)
{
    std::map<int, int> m;
    for (auto &x : in) m[x.first] += x.second;
    std::vector<std::pair<int, int>> out;
    for (auto &x : m) out.push_back(x);
    return out;
}

void parse(Mech &m, const std::string &text)
{
    std::istringstream in(text);
    std::string raw;
    int line = 0, nsp = 0, nth = 0, nrx = 0;
    bool header = false;
    std::vector<bool> have_thermo;
    Reaction *last = nullptr;
    auto need = [&](size_t have, size_t want) {
        if (have < want) throw ParseError("line " + std::to_string(line) + ": too few fields");
    };
    while (std::getline(in, raw)) {
        ++line;
        auto hash = raw.find('#');
        if (hash != std::string::npos) raw.resize(hash);
        std::istringstream ls(raw);
        std::vector<std::string> t;
        for (std::string w; ls >> w;) t.push_back(w);
        if (t.empty()) continue;
        const std::string &key = t[0];
        if (key == "STIFFCHEM-MECH") {
            need(t.size(), 2);
            if (t[1] != "1") throw ParseError("unsupported format version " + t[1]);
            header = true;
        } else if (!header) {
            throw ParseError("line " + std::to_string(line) + ": missing STIFFCHEM-MECH header");
        } else if (key == "NAME") {
            m.name = t.size() > 1 ? t[1] : "";
        } else if (key == "GAS_CONSTANT") {
            need(t.size(), 2);
            m.Rgas = to_double(t[1], line);
        } else if (key == "REF_PRESSURE") {
            need(t.size(), 2);
            m.p0 = to_double(t[1], line);
        } else if (key == "ELEMENTS") {
            need(t.size(), 2);
            m.E = to_int(t[1], line);
            need(t.size(), 2 + (size_t)m.E);
            m.elements.assign(t.begin() + 2, t.begin() + 2 + m.E);
        } else if (key == "SPECIES") {
            need(t.size(), 2);
            m.N = to_int(t[1], line);
            if (m.N <= 0) throw ParseError("species count must be positive");
            m.names.resize(m.N);
            m.W.resize(m.N);
            m.comp.assign((size_t)m.N * std::max(m.E, 1), 0);
            m.nasa.assign((size_t)m.N * 7, 0.0);
            have_thermo.assign(m.N, false);
        } else if (key == "SP") {
            if (nsp >= m.N) throw ParseError("line " + std::to_string(line) + ": more SP lines than SPECIES");
            need(t.size(), 3 + (size_t)m.E);
            if (m.species(t[1]) >= 0) throw ParseError("duplicate species " + t[1]);
            m.names[nsp] = t[1];
            m.W[nsp] = to_double(t[2], line);
            if (!(m.W[nsp] > 0)) throw ParseError("species " + t[1] + ": molar mass must be positive");
            for (int e = 0; e < m.E; ++e) {
                m.comp[nsp * m.E + e] = to_int(t[3 + e], line);
                if (m.comp[nsp * m.E + e] < 0) throw ParseError("negative element count");
            }
            ++nsp;
        } else if (key == "NASA7") {
            need(t.size(), 9);
            int k = m.species(t[1]);
            if (k < 0) throw ParseError("line " + std::to_string(line) + ": NASA7 for unknown species " + t[1]);
            for (int i = 0; i < 7; ++i) m.nasa[k * 7 + i] = to_double(t[2 + i], line);
            if (have_thermo[k]) throw ParseError("duplicate NASA7 for " + t[1]);
            have_thermo[k] = true;
            ++nth;
        } else if (key == "REACTIONS") {
            need(t.size(), 2);
            m.R = to_int(t[1], line);
            if (m.R <= 0) throw ParseError("reaction count must be positive");
            m.rx.reserve(m.R);
        } else if (key == "RX") {
            if (nrx >= m.R) throw ParseError("line " + std::to_string(line) + ": more RX lines than REACTIONS");
            need(t.size(), 7);
            Reaction r;
            if (t[1] == "plain") r.kind = RX_PLAIN;
            else if (t[1] == "third") r.kind = RX_THIRD;
            else if (t[1] == "troe") r.kind = RX_TROE;
            else throw ParseError("line " + std::to_string(line) + ": unknown reaction kind " + t[1]);
            r.log10A = to_double(t[2], line);
            r.b = to_double(t[3], line);
            r.Ea = to_double(t[4], line);
            size_t p = 5;
            for (int side = 0; side < 2; ++side) {
                need(t.size(), p + 1);
                int cnt = to_int(t[p++], line);
                if (cnt < 1) throw ParseError("line " + std::to_string(line) + ": empty reaction side");
                std::vector<std::pair<int, int>> lst;
                for (int i = 0; i < cnt; ++i) {
                    need(t.size(), p + 2);
                    int k = m.species(t[p]);
                    if (k < 0) throw ParseError("line " + std::to_string(line) + ": unknown species " + t[p]);
                    int nu = to_int(t[p + 1], line);
                    if (nu < 1 || nu > 3) throw ParseError("line " + std::to_string(line) + ": stoichiometric coefficient must be 1..3");
                    lst.push_back({k, nu});
                    p += 2;
                }
                (side == 0 ? r.reac : r.prod) = merge_side(lst);
            }
            if (p != t.size()) throw ParseError("line " + std::to_string(line) + ": trailing fields");
            m.rx.push_back(r);
            last = &m.rx.back();
            ++nrx;
        } else if (key == "EFF") {
            if (!last || last->kind == RX_PLAIN) throw ParseError("line " + std::to_string(line) + ": EFF must follow a third/troe RX");
            need(t.size(), 2);
            int cnt = to_int(t[1], line);
            need(t.size(), 2 + 2 * (size_t)cnt);
            for (int i = 0; i < cnt; ++i) {
                int k = m.species(t[2 + 2 * i]);
                if (k < 0) throw ParseError("line " + std::to_string(line) + ": unknown species " + t[2 + 2 * i]);
                double a = to_double(t[3 + 2 * i], line);
                if (a < 0) throw ParseError("negative third-body efficiency");
                for (auto &x : last->eff)
                    if (x.first == k)
                        throw ParseError("line " + std::to_string(line) + ": duplicate efficiency for species " +
                                         t[2 + 2 * i]);
                last->eff.push_back({k, a});
            }
        } else if (key == "TROE") {
            if (!last || last->kind != RX_TROE) throw ParseError("line " + std::to_string(line) + ": TROE must follow a troe RX");
            need(t.size(), 8);
            for (int i = 0; i < 7; ++i) last->troe[i] = to_double(t[1 + i], line);
            if (!(last->troe[4] > 0 && last->troe[5] > 0 && last->troe[6] > 0))
                throw ParseError("Troe temperatures must be positive");
            last->troe[6] = last->troe[6];
        } else if (key == "END") {
            break;
        } else {
            throw ParseError("line " + std::to_string(line) + ": unknown keyword " + key);
        }
    }
    if (!header) throw ParseError("missing STIFFCHEM-MECH header");
    if (m.N <= 0 || nsp != m.N) throw ParseError("species list incomplete");
    if (nth != m.N) throw ParseError("NASA7 data missing for some species");
    if (m.R <= 0 || nrx != m.R) throw ParseError("reaction list incomplete");
}

void validate(Mech &m)
{
    for (int j = 0; j < m.R; ++j) {
        const Reaction &r = m.rx[j];
        for (int e = 0; e < m.E; ++e) {
            long bal = 0;
            for (auto &x : r.reac) bal -= (long)x.second * m.comp[x.first * m.E + e];
            for (auto &x : r.prod) bal += (long)x.second * m.comp[x.first * m.E + e];
            if (bal != 0)
                throw ParseError("reaction " + std::to_string(j) + " does not balance element " + m.elements[e]);
        }
        // coefficients after repeated species on a side are merged: the
        // kernels raise concentrations to integer powers 1..3 only
        for (const auto *side : {&r.reac, &r.prod})
            for (auto &x : *side)
                if (x.second > 3)
                    throw Unsupported("reaction " + std::to_string(j) + ": species " + m.names[x.first] +
                                      " has a merged stoichiometric coefficient above 3");
        if ((int)r.reac.size() > MAXSIDE || (int)r.prod.size() > MAXSIDE)
            throw Unsupported("reaction " + std::to_string(j) + ": more than 3 distinct species on a side");
        int enh = 0;
        for (auto &x : r.eff)
            if (x.second != 1.0) ++enh;
        if (enh > MAXENH)
            throw Unsupported("reaction " + std::to_string(j) + ": more than 4 enhanced third-body species");
        if (r.kind == RX_TROE && r.troe[3] == 0 && r.troe[4] <= 0)
            throw ParseError("bad Troe parameters");
    }
    if (m.N + 1 > MAX_STATE_SPARSE)
        throw Unsupported("mechanism has " + std::to_string(m.N) + " species; the kernels support up to " +
                          std::to_string(MAX_STATE_SPARSE - 1));
}

void build_tables(Mech &m)
{
    Tables &T = m.tab;
    const int N = m.N, R = m.R;
    T.N = N;
    T.R = R;
    T.Rgas = m.Rgas;
    T.p0 = m.p0;
    T.W = m.W;
    T.invW.resize(N);
    T.nasa.resize(7 * N);
    for (int k = 0; k < N; ++k) {
        T.invW[k] = 1.0 / m.W[k];
        for (int c = 0; c < 7; ++c) T.nasa[c * N + k] = m.nasa[k * 7 + c];
    }
    auto rs = [&](std::vector<int32_t> &v, int fill) { v.assign((size_t)MAXSIDE * R, fill); };
    T.kind.resize(R);
    T.nr.resize(R);
    T.np.resize(R);
    T.dnu.resize(R);
    T.neff.resize(R);
    T.tix.assign(R, -1);
    rs(T.rsp, 0);
    rs(T.rnu, 0);
    rs(T.psp, 0);
    rs(T.pnu, 0);
    T.esp.assign((size_t)MAXENH * R, 0);
    T.eam1.assign((size_t)MAXENH * R, 0.0);
    T.lnA.resize(R);
    T.b.resize(R);
    T.EaR.resize(R);
    std::vector<int> troe_ids;
    const double LN10 = std::log(10.0);
    m.n_third = m.n_troe = 0;
    for (int j = 0; j < R; ++j) {
        const Reaction &r = m.rx[j];
        T.kind[j] = r.kind;
        T.nr[j] = (int)r.reac.size();
        T.np[j] = (int)r.prod.size();
        int order = 0, dnu = 0;
        for (size_t i = 0; i < r.reac.size(); ++i) {
            T.rsp[i * R + j] = r.reac[i].first;
            T.rnu[i * R + j] = r.reac[i].second;
            order += r.reac[i].second;
            dnu -= r.reac[i].second;
        }
        for (size_t i = 0; i < r.prod.size(); ++i) {
            T.psp[i * R + j] = r.prod[i].first;
            T.pnu[i * R + j] = r.prod[i].second;
            dnu += r.prod[i].second;
        }
        T.dnu[j] = dnu;
        int n = 0;
        for (auto &x : r.eff)
            if (x.second != 1.0) {
                T.esp[n * R + j] = x.first;
                T.eam1[n * R + j] = x.second - 1.0;
                ++n;
            }
        T.neff[j] = r.kind == RX_PLAIN ? 0 : n;
        // cgs -> SI: A [(cm^3/mol)^(m-1)/s] * 1e-6^(m-1), m = reaction order
        int m_inf = order + (r.kind == RX_THIRD ? 1 : 0);
        T.lnA[j] = r.log10A * LN10 - 6.0 * (m_inf - 1) * LN10;
        T.b[j] = r.b;
        T.EaR[j] = r.Ea / m.Rgas;
        if (r.kind == RX_THIRD) ++m.n_third;
        if (r.kind == RX_TROE) {
            T.tix[j] = (int)troe_ids.size();
            troe_ids.push_back(j);
            ++m.n_troe;
        }
    }
    const int nt = (int)troe_ids.size();
    T.n_troe = nt;
    T.troe.assign((size_t)8 * std::max(nt, 1), 0.0);
    for (int t = 0; t < nt; ++t) {
        const Reaction &r = m.rx[troe_ids[t]];
        int order = 0;
        for (auto &x : r.reac) order += x.second;
        T.troe[0 * nt + t] = r.troe[0] * LN10 - 6.0 * order * LN10;  // k0 is one order higher
        T.troe[1 * nt + t] = r.troe[1];
        T.troe[2 * nt + t] = r.troe[2] / m.Rgas;
        T.troe[3 * nt + t] = r.troe[3];
        T.troe[4 * nt + t] = 1.0 / r.troe[4];
        T.troe[5 * nt + t] = 1.0 / r.troe[5];
        T.troe[6 * nt + t] = r.troe[6];
    }
}

void count_work(Mech &m)
{
    const int N = m.N, R = m.R, n = N + 1;
    Counts &c = m.cnt;
    // structural pattern of the sparse analytical terms (species block, T
    // row and column); the rank-one density coupling makes J itself dense
    std::vector<uint8_t> pat((size_t)n * n, 0);
    for (int i = 0; i < n; ++i) {
        pat[i * n + i] = 1;
        pat[i * n + N] = 1;
        pat[N * n + i] = 1;
    }
    int64_t f_rx = 0, f_jrx = 0;
    int exps = 1;  // log T
    for (int j = 0; j < R; ++j) {
        const Reaction &r = m.rx[j];
        std::vector<int> rows, deps;
        for (auto &x : r.reac) rows.push_back(x.first), deps.push_back(x.first);
        for (auto &x : r.prod) rows.push_back(x.first), deps.push_back(x.first);
        if (r.kind != RX_PLAIN)
            for (auto &x : r.eff)
                if (x.second != 1.0) deps.push_back(x.first);
        for (int a : rows)
            for (int b : deps) pat[a * n + b] = 1;
        const int ns = (int)(r.reac.size() + r.prod.size());
        int nu_tot = 0;
        for (auto &x : r.reac) nu_tot += x.second;
        for (auto &x : r.prod) nu_tot += x.second;
        // kinf (4), lnKc (2 per species + 3), kr (2), products (nu_tot),
        // q (3), scatter (2 per species)
        f_rx += 4 + 2 * ns + 3 + 2 + nu_tot + 3 + 2 * ns;
        exps += 2;
        if (r.kind == RX_THIRD) f_rx += 3 + 2 * (int)deps.size();
        if (r.kind == RX_TROE) {
            f_rx += 4 + 2 * (int)deps.size() + 30;
            exps += 1 + 3 + 2 + 1;  // k0, Fcent (3 exp), 2 log10, 10^x
        }
        const int nd = (int)deps.size();
        // derivative slots (3 each), T derivative (10), euler (2 nd),
        // scatter rows x (deps + T) + T row + u (2 flops each)
        f_jrx += 3 * nd + 10 + 2 * nd + 2 * (ns * (nd + 1) + nd + 1 + ns);
        if (r.kind == RX_TROE) f_jrx += 40;
    }
    int nnz = 0;
    for (auto v : pat) nnz += v;
    c.nnz_jac = nnz;
    c.nnz_lu = n * n;
    c.exp_per_rhs = exps;
    const int64_t f_thermo = 31 * (int64_t)N, f_mix = 8 * (int64_t)N, f_fin = 6 * (int64_t)N + 4;
    c.flops_rhs = f_thermo + f_mix + f_rx + f_fin;
    c.flops_jac_terms = f_jrx + 10 * (int64_t)N;
    c.flops_jac = c.flops_rhs + c.flops_jac_terms + 6 * (int64_t)n * n;
    int64_t lu = 0;
    for (int k = 0; k < n; ++k) lu += (n - k - 1) + 2LL * (n - k - 1) * (n - k - 1);
    c.flops_lu = lu;
    c.flops_solve = 2LL * n * (n - 1) + n;
    // one attempt: build M (n^2 + n), LU, 2 new right-hand sides, 4 solves,
    // stage combinations and error norm (~16 n)
    c.flops_attempt = (int64_t)n * n + n + c.flops_lu + 2 * c.flops_rhs + 4 * c.flops_solve + 16LL * n;
    c.flops_accept = c.flops_jac;
    c.flops_step = c.flops_attempt + c.flops_accept;
}

}  // namespace

Mech load_mechanism(const std::string &text)
{
    Mech m;
    parse(m, text);
    validate(m);
    build_tables(m);
    count_work(m);
    compile_sparse(m);
    const int n = m.N + 1;
    // register rows per cell of the dense kernels; above 64 only the sparse
    // kernels (two state components per lane) apply
    m.n_padded = n <= 16 ? 16 : n <= 32 ? 32 : n <= 56 ? 56 : n <= 64 ? 64 : 128;
    return m;
}

}  // namespace sc
