"""CPU tests of the mechanism compiler's sparse algebra (host only): the
species-term pattern against complex-step Jacobians of the oracle, the
bordered system's static LU and solve schedules replayed in NumPy (level by
level, in shuffled item order) against numpy.linalg.solve, the exact work
of the schedule against a counted replay, and the per-reaction entry
indices against the pattern."""
import numpy as np
import pytest

import paper_2311_14941_amd as sc
from oracle.oracle import Oracle
from synth.cells import make_cells
from synth.mechgen import standard_mechanism


@pytest.fixture(scope="module", autouse=True)
def built():
    sc.ensure_built()


_M = {}


def mech(key):
    if key not in _M:
        m = standard_mechanism(key)
        _M[key] = (m, sc.Mechanism(m.to_text()))
    return _M[key]


def arrays(cm):
    names = ("perm", "pattern", "apat", "erow", "ecol", "lu_b_lvl", "lu_c_lvl", "lu_b", "lu_c", "lu_u", "diag",
             "fw_lvl", "bw_lvl", "fw", "bw", "tfw_lvl", "tbw_lvl", "tfw", "tbw", "rxi")
    return {k: cm.sparse_array(k) for k in names}


M16 = np.uint64(0xFFFF)


def lo(x):
    return (x & M16).astype(np.int64)


def mid(x):
    return ((x >> np.uint64(16)) & M16).astype(np.int64)


def hi(x):
    return ((x >> np.uint64(32)) & M16).astype(np.int64)


class Replay:
    """The kernels' schedules executed in NumPy: each level's items at once
    (repeated targets accumulate, as the device's LDS atomics do), items in
    a shuffled order.  Counts the floating-point work it performs."""

    def __init__(self, a, rng, tail):
        self.a, self.rng, self.flops, self.tail = a, rng, 0, tail

    def _shuf(self, x):
        return x[self.rng.permutation(x.size)]

    def lu(self, v):
        a = self.a
        for l in range(a["lu_b_lvl"].size - 1):
            b = self._shuf(a["lu_b"][a["lu_b_lvl"][l]:a["lu_b_lvl"][l + 1]].astype(np.uint64))
            v[lo(b)] = v[lo(b)] / v[mid(b)]
            self.flops += b.size
            c = self._shuf(a["lu_c"][a["lu_c_lvl"][l]:a["lu_c_lvl"][l + 1]])
            np.subtract.at(v, lo(c), v[mid(c)] * v[hi(c)])
            self.flops += 2 * c.size
        # the dense trailing block, eliminated pivot by pivot after the levels
        n = a["perm"].size
        emap = -np.ones((n, n), dtype=np.int64)
        emap[a["erow"], a["ecol"]] = np.arange(a["erow"].size)
        t0 = n - self.tail
        assert np.all(emap[t0:, t0:] >= 0), "the tail block must be full"
        for k in range(t0, n):
            rows = emap[k + 1:, k]
            v[rows] = v[rows] / v[emap[k, k]]
            self.flops += rows.size
            blk = emap[k + 1:, k + 1:]
            v[blk] -= np.outer(v[rows], v[emap[k, k + 1:]])
            self.flops += 2 * blk.size
        d = a["diag"].astype(np.int64)
        dinv = 1.0 / v[d]
        self.flops += d.size
        u = a["lu_u"].astype(np.uint64)
        v[lo(u)] *= dinv[mid(u)]
        self.flops += u.size
        return dinv

    def _sweep(self, lvl, items, v, x):
        for l in range(lvl.size - 1):
            it = self._shuf(items[lvl[l]:lvl[l + 1]])
            np.subtract.at(x, lo(it), v[hi(it)] * x[mid(it)])
            self.flops += 2 * it.size

    def solve(self, v, dinv, x):
        a = self.a
        self._sweep(a["fw_lvl"], a["fw"], v, x)
        x *= dinv
        self.flops += x.size
        self._sweep(a["bw_lvl"], a["bw"], v, x)
        return x

    def solve_t(self, v, dinv, x):
        a = self.a
        self._sweep(a["tfw_lvl"], a["tfw"], v, x)
        x *= dinv
        self._sweep(a["tbw_lvl"], a["tbw"], v, x)
        return x


@pytest.mark.parametrize("key", ["h2_9", "chon_53", "chon_110"])
def test_schedule_solves_like_numpy(key):
    """Random values on the bordered pattern (diagonally dominant, so no
    pivoting is needed): the replayed LU + solves equal numpy.linalg.solve
    for A x = b and A^T w = c.  A missing fill entry, a wrong level or a
    mis-encoded item changes the result."""
    _, cm = mech(key)
    a = arrays(cm)
    n = a["perm"].size
    rng = np.random.default_rng(4)
    P = a["apat"].reshape(n, n).astype(bool)
    er, ec = a["erow"], a["ecol"]
    for trial in range(3):
        A = np.where(P, rng.normal(size=(n, n)), 0.0)
        A[np.arange(n), np.arange(n)] = n + rng.uniform(1, 2, n)
        v = A[er, ec].copy()  # fill entries start at zero
        r = Replay(a, rng, cm.info["lu_tail_sparse"])
        dinv = r.lu(v)
        b = rng.normal(size=n)
        x = r.solve(v, dinv, b.copy())
        assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-12, atol=1e-12 * np.abs(x).max())
        w = r.solve_t(v, dinv, b.copy())
        assert np.allclose(w, np.linalg.solve(A.T, b), rtol=1e-12, atol=1e-12 * np.abs(w).max())


@pytest.mark.parametrize("key", ["h2_9", "chon_53"])
def test_table_sweeps_solve_like_numpy(key):
    """The solves of the several-cells-per-wave kernels, replayed from their
    per-column row tables alone ("sweep_fi", "sweep_bi": the entry of each
    row below / above the diagonal, or nnz, a slot holding zero) on the
    factors of the schedule replay: equal to numpy.linalg.solve.  A wrong
    or missing table entry changes the result."""
    _, cm = mech(key)
    a = arrays(cm)
    n = a["perm"].size
    nnz = a["erow"].size
    fi = cm.sparse_array("sweep_fi").astype(np.int64).reshape(n, 64)
    bi = cm.sparse_array("sweep_bi").astype(np.int64).reshape(n, 64)
    assert np.all(fi[:, n:] == nnz) and np.all(bi[:, n:] == nnz)
    rng = np.random.default_rng(9)
    P = a["apat"].reshape(n, n).astype(bool)
    for trial in range(3):
        A = np.where(P, rng.normal(size=(n, n)), 0.0)
        A[np.arange(n), np.arange(n)] = n + rng.uniform(1, 2, n)
        v = A[a["erow"], a["ecol"]].copy()
        dinv = Replay(a, rng, cm.info["lu_tail_sparse"]).lu(v)
        v = np.append(v, 0.0)  # the zero slot
        b = rng.normal(size=n)
        z = b.copy()
        for k in range(n - 1):  # every lane applies column k at once
            z -= v[fi[k, :n]] * z[k]
        z *= dinv
        for k in range(n - 1, 0, -1):
            z -= v[bi[k, :n]] * z[k]
        assert np.allclose(z, np.linalg.solve(A, b), rtol=1e-12, atol=1e-12 * np.abs(z).max())


@pytest.mark.parametrize("key,width", [("h2_9", 9), ("chon_53", 30), ("chon_110", 64)])
def test_dense_tail_is_the_widest_full_block(key, width):
    """The register-factorised tail is the widest trailing block of the
    filled L+U pattern that is full, capped at 32 positions for systems of
    up to 64 positions and at 64 beyond, and the level schedule holds
    exactly the pivots before it."""
    _, cm = mech(key)
    a = arrays(cm)
    n = a["perm"].size
    w = cm.info["lu_tail_sparse"]
    assert w == width
    F = np.zeros((n, n), dtype=bool)
    F[a["erow"], a["ecol"]] = True
    t0 = n - w
    assert F[t0:, t0:].all()
    assert w == (32 if n <= 64 else 64) or t0 == 0 or not F[t0 - 1:, t0 - 1:].all()
    # b items: the L entries of the scheduled pivots (columns before t0)
    piv = a["ecol"][lo(a["lu_b"].astype(np.uint64))]
    assert np.all(piv < t0) and a["lu_b"].size == int(np.sum((a["erow"] > a["ecol"]) & (a["ecol"] < t0)))


@pytest.mark.parametrize("key", ["h2_9", "chon_53", "chon_110"])
def test_schedule_work_equals_counted_replay(key):
    """flops_lu_sparse and flops_solve_sparse (mechanism info, the roofline's
    numerator) equal the operations a replay of the schedule performs (plus
    the solve's 2N for scaling the species by 1/W and back)."""
    m, cm = mech(key)
    a = arrays(cm)
    n = a["perm"].size
    rng = np.random.default_rng(5)
    A = np.where(a["apat"].reshape(n, n).astype(bool), rng.normal(size=(n, n)), 0.0) + n * np.eye(n)
    v = A[a["erow"], a["ecol"]].copy()
    r = Replay(a, rng, cm.info["lu_tail_sparse"])
    dinv = r.lu(v)
    assert r.flops == cm.info["flops_lu_sparse"]
    r.flops = 0
    r.solve(v, dinv, rng.normal(size=n))
    assert r.flops + 2 * m.n_species == cm.info["flops_solve_sparse"]
    w = cm.info["lu_tail_sparse"]
    assert cm.info["lu_updates_sparse"] == a["lu_c"].size + sum(q * q for q in range(w))
    assert cm.info["nnz_lu_sparse"] == a["erow"].size
    # the ordering is a permutation with the borders (T, sigma) last
    assert sorted(a["perm"]) == list(range(n)) and list(a["perm"][-2:]) == [n - 2, n - 1]


@pytest.mark.parametrize("key,nstates", [("h2_9", 400), ("chon_53", 150), ("chon_110", 80)])
def test_species_pattern_covers_complex_step_jacobian(key, nstates):
    """At constant pressure the species block of the Jacobian is
    J_km = (W_k/W_m) P_km + g_k / W_m (the second term from the density),
    so X_km = (W_m/W_k) J_km equals one value per row for every m outside
    the pattern of P.  On random states the oracle's complex-step Jacobian
    (exact to roundoff) must show that; an entry missing from the pattern
    breaks it.  The check has power: dropping a pattern entry that a
    reaction does feed fails it."""
    m, cm = mech(key)
    a = arrays(cm)
    N = m.n_species
    pat = a["pattern"].reshape(N, N).astype(bool)
    o = Oracle(m.to_text())
    W = m.molar_masses()
    rng = np.random.default_rng(7)
    worst = 0.0
    Xs = []
    for _ in range(nstates):
        Y = rng.dirichlet(np.full(N, 0.3))
        T = rng.uniform(700.0, 2600.0)
        p = 101325.0 * 10 ** rng.uniform(0, 1)
        J = o.jac_cs(np.append(Y, T), p)
        X = J[:N, :N] * W[None, :] / W[:, None]
        Xs.append(X)
        for k in range(N):
            out = X[k, ~pat[k]]
            if out.size < 2:
                continue
            spread = out.max() - out.min()
            worst = max(worst, spread / (np.abs(X[k]).max() + 1e-300))
    assert worst < 1e-9, worst
    # power: remove an in-pattern off-diagonal entry and the spread appears
    rows, cols = np.nonzero(pat & ~np.eye(N, dtype=bool))
    hit = applicable = 0
    for t in rng.permutation(rows.size)[:60]:
        k, mm = rows[t], cols[t]
        if (~pat[k]).sum() < 1:
            continue  # a full row: nothing outside the pattern to compare with
        applicable += 1
        for X in Xs:
            out = X[k, ~pat[k]]
            # the row's own roundoff: the spread of its out-of-pattern values
            noise = max(out.max() - out.min(), 1e-15 * np.abs(X[k]).max())
            if abs(X[k, mm] - out.mean()) > 1e3 * noise:
                hit += 1
                break
    # (a few pattern entries stay negligible at every sampled state: reactions
    # with large activation energies at the lower temperatures)
    assert applicable >= 5 and hit >= 0.6 * applicable, (hit, applicable)


@pytest.mark.parametrize("key", ["h2_9", "chon_53", "chon_110"])
def test_reaction_entry_indices(key):
    """Each reaction's scatter targets are the L+U entries of (its row
    species, its dependency species) and (row, T), (T, dependency), (T, T),
    in positions; unused slots hold 0xFFFF."""
    m, cm = mech(key)
    a = arrays(cm)
    N, n = m.n_species, a["perm"].size
    pos = np.empty(n, np.int64)
    pos[a["perm"]] = np.arange(n)
    rxi = a["rxi"].reshape(m.n_reactions, -1).astype(np.int64)
    NDEP, ROW = 10, 11
    pT = pos[N]
    for j, r in enumerate(m.reactions):
        dep = [k for k, _ in r.reac] + [-1] * (3 - len(r.reac)) + [k for k, _ in r.prod] + [-1] * (3 - len(r.prod))
        enh = [k for k, al in sorted(r.eff.items()) if al != 1.0] if r.kind != "plain" else []
        dep += enh + [-1] * (4 - len(enh))
        rows = [k for k, _ in r.reac] + [None] * (3 - len(r.reac)) + [k for k, _ in r.prod] + [None] * (3 - len(r.prod))
        for rs, row in enumerate(rows):
            for s in range(NDEP + 1):
                e = rxi[j, rs * ROW + s]
                if row is None or (s < NDEP and dep[s] < 0):
                    assert e == 0xFFFF
                    continue
                col = pT if s == NDEP else pos[dep[s]]
                assert (a["erow"][e], a["ecol"][e]) == (pos[row], col)
        for s in range(NDEP):
            e = rxi[j, 6 * ROW + s]
            if dep[s] < 0:
                assert e == 0xFFFF
            else:
                assert (a["erow"][e], a["ecol"][e]) == (pT, pos[dep[s]])
        e = rxi[j, 6 * ROW + NDEP]
        assert (a["erow"][e], a["ecol"][e]) == (pT, pT)
