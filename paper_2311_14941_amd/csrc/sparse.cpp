// The sparse compile of a mechanism (host side): the structural pattern of
// the analytical Jacobian terms, a minimum-degree ordering of the species,
// the bordered system, its symbolic LU, the static level schedules of the
// factorisation and of the triangular solves, the entry each reaction's
// derivative terms land in, and the exact work of the schedule.
//
// The paper's chemistry library manages the sparse algebra of the mechanism
// and forms a sparse analytical Jacobian (Sec. 2.5); this is that
// management, done once per mechanism so that the device kernels only
// follow a fixed list of operations.
#include <algorithm>
#include <array>
#include <cstdint>
#include <numeric>
#include <vector>

#include "mech.hpp"

namespace sc {

namespace {

// Reaction j's dependency-slot species (slots as in the device record:
// reactants 0..2, products 3..5, enhanced third-body species 6..9), -1 when
// unused.
void dep_slots(const Reaction &r, int (&dep)[NDEP])
{
    for (int s = 0; s < NDEP; ++s) dep[s] = -1;
    for (size_t i = 0; i < r.reac.size() && i < (size_t)MAXSIDE; ++i) dep[i] = r.reac[i].first;
    for (size_t i = 0; i < r.prod.size() && i < (size_t)MAXSIDE; ++i) dep[MAXSIDE + i] = r.prod[i].first;
    if (r.kind != RX_PLAIN) {
        int e = 0;
        for (auto &x : r.eff)
            if (x.second != 1.0 && e < MAXENH) dep[2 * MAXSIDE + e++] = x.first;
    }
}

// Greedy minimum-degree ordering of the symmetric graph g (n x n adjacency,
// no self loops): repeatedly eliminate a vertex of least current degree
// (lowest index on ties) and join its neighbours into a clique.
std::vector<int> minimum_degree(std::vector<uint8_t> g, int n)
{
    std::vector<int> order;
    std::vector<uint8_t> alive(n, 1);
    for (int step = 0; step < n; ++step) {
        int best = -1, bdeg = 1 << 30;
        for (int v = 0; v < n; ++v) {
            if (!alive[v]) continue;
            int d = 0;
            for (int u = 0; u < n; ++u) d += alive[u] && g[v * n + u];
            if (d < bdeg) bdeg = d, best = v;
        }
        std::vector<int> nb;
        for (int u = 0; u < n; ++u)
            if (alive[u] && g[best * n + u]) nb.push_back(u);
        for (int a : nb)
            for (int b : nb)
                if (a != b) g[a * n + b] = 1;
        alive[best] = 0;
        order.push_back(best);
    }
    return order;
}

// Level of every row of a triangular solve: a row is final once every row
// it reads is final.  reads[i] = rows i depends on.
std::vector<int> solve_levels(const std::vector<std::vector<int>> &reads, const std::vector<int> &seq)
{
    std::vector<int> lev(reads.size(), 0);
    for (int i : seq)
        for (int p : reads[i]) lev[i] = std::max(lev[i], lev[p] + 1);
    return lev;
}

// Items x_target -= value(entry) x_source grouped by the level of their
// source (a source is final after all earlier levels), as offsets + items.
void group_by_source(const std::vector<std::array<int, 3>> &items, const std::vector<int> &lev,
                     std::vector<int> &lvl, std::vector<uint64_t> &out)
{
    int nl = 0;
    for (auto &it : items) nl = std::max(nl, lev[it[1]] + 1);
    std::vector<std::vector<uint64_t>> by(nl);
    for (auto &it : items)
        by[lev[it[1]]].push_back((uint64_t)it[0] | (uint64_t)it[1] << 16 | (uint64_t)it[2] << 32);
    lvl.assign(1, 0);
    out.clear();
    for (auto &b : by) {
        if (b.empty()) continue;
        out.insert(out.end(), b.begin(), b.end());
        lvl.push_back((int)out.size());
    }
}

}  // namespace

void compile_sparse(Mech &m)
{
    const int N = m.N, R = m.R;
    const int n = N + 2;  // species, T, sigma
    SparseLU &S = m.sp;
    S = SparseLU();
    S.n = n;
    // 1. structural pattern of the species terms P_km (plus the diagonal)
    m.pattern.assign((size_t)N * N, 0);
    for (int k = 0; k < N; ++k) m.pattern[k * N + k] = 1;
    for (int j = 0; j < R; ++j) {
        int dep[NDEP];
        dep_slots(m.rx[j], dep);
        for (auto *side : {&m.rx[j].reac, &m.rx[j].prod})
            for (auto &row : *side)
                for (int s = 0; s < NDEP; ++s)
                    if (dep[s] >= 0) m.pattern[row.first * N + dep[s]] = 1;
    }
    // 2. minimum-degree order of the species on the symmetrised pattern
    std::vector<uint8_t> g((size_t)N * N, 0);
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b)
            if (a != b && (m.pattern[a * N + b] || m.pattern[b * N + a])) g[a * N + b] = 1;
    std::vector<int> order = minimum_degree(g, N);
    S.perm = order;
    S.perm.push_back(N);      // T
    S.perm.push_back(N + 1);  // sigma
    S.pos.assign(n, 0);
    for (int q = 0; q < n; ++q) S.pos[S.perm[q]] = q;
    // 3. the bordered pattern in positions
    std::vector<uint8_t> A((size_t)n * n, 0);
    const int pT = S.pos[N], pS = S.pos[N + 1];
    for (int a = 0; a < N; ++a) {
        for (int b = 0; b < N; ++b)
            if (m.pattern[a * N + b]) A[S.pos[a] * n + S.pos[b]] = 1;
        A[S.pos[a] * n + pT] = A[S.pos[a] * n + pS] = 1;  // T and sigma columns
        A[pT * n + S.pos[a]] = A[pS * n + S.pos[a]] = 1;  // T and sigma rows
    }
    A[pT * n + pT] = A[pS * n + pS] = 1;
    S.apat = A;
    for (auto v : A) S.nnz_a += v;
    // 4. symbolic LU: right-looking elimination without pivoting
    std::vector<uint8_t> F = A;
    std::vector<std::vector<int>> Lc(n), Ur(n);  // strict L column k, strict U row k
    for (int k = 0; k < n; ++k) {
        for (int i = k + 1; i < n; ++i)
            if (F[i * n + k]) Lc[k].push_back(i);
        for (int j = k + 1; j < n; ++j)
            if (F[k * n + j]) Ur[k].push_back(j);
        for (int i : Lc[k])
            for (int j : Ur[k]) F[i * n + j] = 1;
    }
    // entries numbered column by column, rows ascending within a column, so
    // a column's entries are contiguous: the entry of (i, j) is the column's
    // start plus the number of its rows above i (what the device solves
    // compute from the column's row mask)
    S.emap.assign((size_t)n * n, -1);
    S.cstart.assign(1, 0);
    S.cmask.assign(2 * (size_t)n, 0);
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < n; ++i)
            if (F[i * n + j]) {
                S.emap[i * n + j] = (int)S.erow.size();
                S.erow.push_back(i);
                S.ecol.push_back(j);
                S.cmask[2 * j + i / 64] |= 1ull << (i % 64);
            }
        S.cstart.push_back((int)S.erow.size());
    }
    S.nnz = (int)S.erow.size();
    S.sweep_f.clear();
    S.sweep_b.clear();
    S.sweep_fi.clear();
    S.sweep_bi.clear();
    if (n <= 64) {
        for (int k = 0; k < n; ++k) {
            const uint64_t m = S.cmask[2 * k];
            const uint64_t upto = k == 63 ? ~0ull : (2ull << k) - 1;  // rows 0..k
            const uint64_t lower = m & ~upto, upper = m & ((1ull << k) - 1);
            const uint32_t lstart = (uint32_t)(S.cstart[k] + __builtin_popcountll(m & upto));
            for (uint32_t w : {(uint32_t)lower, (uint32_t)(lower >> 32), lstart, 0u}) S.sweep_f.push_back(w);
            for (uint32_t w : {(uint32_t)upper, (uint32_t)(upper >> 32), (uint32_t)S.cstart[k], 0u})
                S.sweep_b.push_back(w);
        }
        const int nz = (int)S.erow.size();
        S.sweep_fi.assign((size_t)n * 64, (uint16_t)nz);
        S.sweep_bi.assign((size_t)n * 64, (uint16_t)nz);
        for (int k = 0; k < n; ++k)
            for (int e = S.cstart[k]; e < S.cstart[k + 1]; ++e) {
                const int i = S.erow[e];
                if (i > k) S.sweep_fi[(size_t)k * 64 + i] = (uint16_t)e;
                if (i < k) S.sweep_bi[(size_t)k * 64 + i] = (uint16_t)e;
            }
    }
    if (S.nnz >= NOENT) throw Unsupported("sparse LU has too many entries for 16-bit entry indices");
    auto E = [&](int i, int j) { return S.emap[i * n + j]; };
    // 5. the dense trailing block: the widest [t, n) of at most
    //    sparse_tail_max(n) positions whose L+U pattern is full (the trailing
    //    Schur complement of a minimum-degree order fills in).  Its pivots
    //    would take one level each; they are factorised in registers instead,
    //    after the levels of the pivots before t.
    S.tail0 = n;
    while (S.tail0 > 0 && n - S.tail0 < sparse_tail_max(n)) {
        const int q = S.tail0 - 1;
        bool full = true;
        for (int i = q; i < n && full; ++i) full = F[(size_t)i * n + q] && F[(size_t)q * n + i];
        if (!full) break;
        S.tail0 = q;
    }
    // 6. LU levels of the pivots before the tail: pivot k waits for every
    //    earlier pivot that updates its row or column (k in L_p or in U_p);
    //    at least one (possibly empty) level
    std::vector<int> lev(n, 0);
    for (int p = 0; p < n; ++p) {
        for (int i : Lc[p]) lev[i] = std::max(lev[i], lev[p] + 1);
        for (int j : Ur[p]) lev[j] = std::max(lev[j], lev[p] + 1);
    }
    int nl = 1;
    for (int k = 0; k < S.tail0; ++k) nl = std::max(nl, lev[k] + 1);
    S.lu_b_lvl.assign(1, 0);
    S.lu_c_lvl.assign(1, 0);
    int64_t nL = 0, nU = 0;
    for (int l = 0; l < nl; ++l) {
        for (int k = 0; k < S.tail0; ++k) {
            if (lev[k] != l) continue;
            for (int i : Lc[k]) S.lu_b.push_back((uint32_t)E(i, k) | (uint32_t)E(k, k) << 16);
            for (int i : Lc[k])
                for (int j : Ur[k])
                    S.lu_c.push_back((uint64_t)E(i, j) | (uint64_t)E(i, k) << 16 | (uint64_t)E(k, j) << 32);
        }
        S.lu_b_lvl.push_back((int)S.lu_b.size());
        S.lu_c_lvl.push_back((int)S.lu_c.size());
    }
    S.diag.resize(n);
    for (int k = 0; k < n; ++k) {
        S.diag[k] = (uint32_t)E(k, k);
        nL += (int64_t)Lc[k].size();
        nU += (int64_t)Ur[k].size();
        S.updates += (int64_t)Lc[k].size() * (int64_t)Ur[k].size();
        for (int j : Ur[k]) S.lu_u.push_back((uint32_t)E(k, j) | (uint32_t)k << 16);
    }
    // 7. solves.  Forward (unit L): x_i -= l_ip x_p.  Backward (U scaled to a
    //    unit diagonal, after x *= 1/u_kk): x_k -= u'_kj x_j.
    std::vector<std::vector<int>> rd(n);
    std::vector<std::array<int, 3>> items;
    std::vector<int> up(n), down(n);
    std::iota(up.begin(), up.end(), 0);
    std::iota(down.rbegin(), down.rend(), 0);
    for (int p = 0; p < n; ++p)
        for (int i : Lc[p]) rd[i].push_back(p), items.push_back({i, p, E(i, p)});
    group_by_source(items, solve_levels(rd, up), S.fw_lvl, S.fw);
    rd.assign(n, {});
    items.clear();
    for (int k = 0; k < n; ++k)
        for (int j : Ur[k]) rd[k].push_back(j), items.push_back({k, j, E(k, j)});
    group_by_source(items, solve_levels(rd, down), S.bw_lvl, S.bw);
    // transposed: A^T = U'^T D L^T.  Forward with U'^T: y_j -= u'_kj y_k;
    // then y *= 1/u_kk; backward with L^T: w_p -= l_ip w_i
    rd.assign(n, {});
    items.clear();
    for (int k = 0; k < n; ++k)
        for (int j : Ur[k]) rd[j].push_back(k), items.push_back({j, k, E(k, j)});
    group_by_source(items, solve_levels(rd, up), S.tfw_lvl, S.tfw);
    rd.assign(n, {});
    items.clear();
    for (int p = 0; p < n; ++p)
        for (int i : Lc[p]) rd[p].push_back(i), items.push_back({p, i, E(i, p)});
    group_by_source(items, solve_levels(rd, down), S.tbw_lvl, S.tbw);
    // 8. the entries each reaction's derivative terms are scattered into
    S.rxi.assign((size_t)R * RXI_SIZE, NOENT);
    for (int j = 0; j < R; ++j) {
        const Reaction &r = m.rx[j];
        int dep[NDEP];
        dep_slots(r, dep);
        uint16_t *x = &S.rxi[(size_t)j * RXI_SIZE];
        for (int rs = 0; rs < 2 * MAXSIDE; ++rs) {
            const auto &side = rs < MAXSIDE ? r.reac : r.prod;
            const int ri = rs % MAXSIDE;
            if (ri >= (int)side.size()) continue;
            const int row = S.pos[side[ri].first];
            for (int s = 0; s < NDEP; ++s)
                if (dep[s] >= 0) x[rs * RXI_ROW + s] = (uint16_t)E(row, S.pos[dep[s]]);
            x[rs * RXI_ROW + NDEP] = (uint16_t)E(row, pT);
        }
        for (int s = 0; s < NDEP; ++s)
            if (dep[s] >= 0) x[RXI_TROW + s] = (uint16_t)E(pT, S.pos[dep[s]]);
        x[RXI_TROW + NDEP] = (uint16_t)E(pT, pT);
    }
    S.e_kk.resize(N);
    S.e_kT.resize(N);
    S.e_kS.resize(N);
    S.e_Tk.resize(N);
    S.e_Sk.resize(N);
    for (int k = 0; k < N; ++k) {
        const int q = S.pos[k];
        S.e_kk[k] = E(q, q);
        S.e_kT[k] = E(q, pT);
        S.e_kS[k] = E(q, pS);
        S.e_Tk[k] = E(pT, q);
        S.e_Sk[k] = E(pS, q);
    }
    S.e_TT = E(pT, pT);
    S.e_SS = E(pS, pS);
    S.e_TS = E(pT, pS);
    S.e_ST = E(pS, pT);
    // 9. work of the schedule (fma = 2 flops, division = 1): LU = one division
    //    per L entry, one fma per Schur update, the reciprocal of every pivot
    //    and the row scaling of U; a solve = the scaled right-hand side (1/W_k
    //    per species), one fma per L and U entry, the pivot scaling, and the
    //    unscaling of the species (W_k)
    S.flops_lu = nL + 2 * S.updates + n + nU;
    S.flops_solve = 2 * nL + 2 * nU + n + 2LL * N;
    Counts &c = m.cnt_sparse;
    c = m.cnt;
    const int ns = N + 1;
    c.nnz_lu = S.nnz;
    c.flops_lu = S.flops_lu;
    c.flops_solve = S.flops_solve;
    // the Jacobian pass: right-hand side, derivative terms and the border
    // formation (about 20 flops per state component)
    c.flops_jac = c.flops_rhs + c.flops_jac_terms + 20LL * ns;
    c.flops_attempt = ns + c.flops_lu + 2 * c.flops_rhs + 4 * c.flops_solve + 16LL * ns;
    c.flops_accept = c.flops_jac;
    c.flops_step = c.flops_attempt + c.flops_accept;
}

}  // namespace sc
