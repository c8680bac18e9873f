"""CPU pins of the operator-split driver's reference (oracle/split.py) and
of the synthetic flame field.

The transport update is pinned by closed forms: at Co = 1 and D = 0 it is an
exact shift by one cell (upwind direction, inflow column); without
advection the cosine modes of the zero-gradient grid are its eigenvectors
with the factor 1 - 4 Fo sin^2(pi k / 2n) per direction; with zero boundary
flux it conserves the sum; with Co + 4 Fo <= 1 it obeys the maximum
principle.  The split step's order (chemistry, then transport) is pinned
by a shift: after one step at Co = 1 a cell holds its west neighbour's
reacted state."""
import numpy as np
import pytest

from oracle.split import split_run, transport2d


def _rand(rng, ncomp, nx, ny):
    return rng.uniform(0.1, 2.0, (ncomp, nx * ny)), rng.uniform(0.1, 2.0, (ncomp, ny))


def test_constant_field_is_fixed():
    nx, ny = 7, 5
    q = np.full((3, nx * ny), 0.37)
    inflow = np.full((3, ny), 0.37)
    rng = np.random.default_rng(1)
    u = rng.uniform(0, 10, nx * ny)
    dt = np.full(nx * ny, 1e-5)
    out = transport2d(q, u, dt, 1e-3, 1e-2, inflow, nx, ny)
    assert np.abs(out - 0.37).max() < 1e-15


def test_unit_courant_advection_is_a_shift():
    nx, ny, dx = 9, 4, 2e-3
    rng = np.random.default_rng(2)
    q, inflow = _rand(rng, 2, nx, ny)
    u = np.full(nx * ny, 5.0)
    dt = np.full(nx * ny, dx / 5.0)
    out = transport2d(q, u, dt, dx, 0.0, inflow, nx, ny).reshape(2, ny, nx)
    g = q.reshape(2, ny, nx)
    # exact up to the rounding of q - (q - q_W) and of Co itself
    assert np.allclose(out[:, :, 1:], g[:, :, :-1], rtol=1e-15, atol=0)
    assert np.allclose(out[:, :, 0], inflow, rtol=1e-15, atol=0)


@pytest.mark.parametrize("axis,k", [(0, 1), (0, 3), (1, 2), (1, 5)])
def test_diffusion_cosine_modes(axis, k):
    nx, ny, dx, D = 12, 10, 1e-3, 3e-2
    dt = 0.2 * dx * dx / D                       # Fo = 0.2
    ix, iy = np.meshgrid(np.arange(nx), np.arange(ny))
    if axis == 0:
        f = np.cos(np.pi * k * (iy + 0.5) / ny)
        n = ny
    else:
        f = np.cos(np.pi * k * (ix + 0.5) / nx)
        n = nx
    q = f.reshape(1, -1)
    inflow = f[:, 0][None, :]                    # west ghost = mirror of column 0
    out = transport2d(q, np.zeros(nx * ny), np.full(nx * ny, dt), dx, D, inflow, nx, ny)
    lam = 1.0 - 4.0 * 0.2 * np.sin(np.pi * k / (2 * n)) ** 2
    assert np.allclose(out, lam * q, rtol=0, atol=1e-14)


def test_zero_flux_diffusion_conserves_sum():
    nx, ny = 11, 8
    rng = np.random.default_rng(3)
    q, _ = _rand(rng, 3, nx, ny)
    inflow = q.reshape(3, ny, nx)[:, :, 0].copy()
    # one dt for all cells: with local steps the two sides of a face use
    # different dt, and the update conserves only at steady state
    dt = np.full(nx * ny, 2.0e-5)                 # Fo = 0.2
    out = transport2d(q, np.zeros(nx * ny), dt, 1e-3, 1e-2, inflow, nx, ny)
    assert abs(out.sum() - q.sum()) < 1e-12 * q.sum()


def test_maximum_principle_and_mass_fraction_sum():
    nx, ny, dx, D = 13, 9, 1e-3, 2e-4
    rng = np.random.default_rng(4)
    Y = rng.dirichlet(np.ones(5), nx * ny).T
    inflow = rng.dirichlet(np.ones(5), ny).T
    u = rng.uniform(0, 40, nx * ny)
    dt = rng.uniform(0.2, 1.0, nx * ny) * 0.5 * np.minimum(dx / u, dx * dx / (4 * D))
    out = transport2d(Y, u, dt, dx, D, inflow, nx, ny)
    lo = min(Y.min(), inflow.min())
    hi = max(Y.max(), inflow.max())
    assert out.min() >= lo - 1e-15 and out.max() <= hi + 1e-15
    assert np.abs(out.sum(0) - 1.0).max() < 1e-14


def test_split_step_is_chemistry_then_transport():
    from oracle.oracle import Oracle
    from synth.cells import make_cells
    c = make_cells("C1", n=8, seed=9)
    o = Oracle(c["mech"].to_text())
    nx, ny, dx = 4, 2, 1e-3
    field = dict(T=c["T"], p=c["p"], Y=c["Y"], u=np.full(8, 10.0), dt=np.full(8, dx / 10.0), dx=dx, D=0.0,
                 nx=nx, ny=ny, inflow_T=np.array([300.0, 310.0]), inflow_Y=c["Y"][[0, 4]].T.copy())
    T1, Y1, st = split_run(o, field, 1, rtol=1e-8, atol=1e-14)
    assert np.all(st[0] == 0)
    r = o.integrate(c["T"], c["p"], c["Y"], field["dt"], rtol=1e-8, atol=1e-14)
    g = np.arange(8).reshape(ny, nx)
    for iy in range(ny):
        assert np.isclose(T1[g[iy, 0]], field["inflow_T"][iy], rtol=1e-15, atol=0)
        for ix in range(1, nx):
            assert np.isclose(T1[g[iy, ix]], r["T"][g[iy, ix - 1]], rtol=1e-15, atol=0)
            assert np.allclose(Y1[g[iy, ix]], r["Y"][g[iy, ix - 1]], rtol=1e-15, atol=1e-17)


def test_flame_field_structure():
    from synth.field import flame_field
    f = flame_field()
    n = f["nx"] * f["ny"]
    assert n == 28900 and f["Y"].shape == (n, f["N"])
    assert np.abs(f["Y"].sum(1) - 1).max() < 1e-14 and f["Y"].min() >= 0
    assert set(np.unique(f["stream"])) == {0, 1, 2}
    co = f["u"] * f["dt"] / f["dx"]
    fo = f["D"] * f["dt"] / f["dx"] ** 2
    assert np.all(co + 4 * fo <= 1.0) and np.all(f["dt"] > 0)
    # the local steps span the CFL range of the jet and the coflow
    assert f["dt"].max() / f["dt"].min() > 20
    assert np.all(f["T"][f["stream"] == 1] == 1880.0)
