"""Seeded synthetic 2-D jet-flame field for the operator-split driver (input
generator only: no chemistry arithmetic of the method lives here).

The paper's flame runs on about 29,000 cells of a 2-D grid (Table 1) around
a 7.2 mm fuel jet surrounded by a pilot (7.7-18.2 mm) and a coflow (Fig. 1),
with a local time step per cell (Sec. 2.5).  This field reproduces that
structure on a uniform nx x ny grid of the 53-species mechanism:

* streams by |y|: jet (|y| < 3.6 mm) a methane/ammonia/air mixture at 294 K,
  pilot (3.85-9.1 mm) burnt gas at 1880 K (the Gibbs minimum of a lean
  mixture's elements at that temperature), coflow air at 291 K;
* axial velocity u(x, y) = Uc + (Uj - Uc) b0/b(x) exp(-(y/b(x))^2) with
  b(x) = b0 + 0.08 x (a spreading jet), Uj = 49.6 m/s, Uc = 0.9 m/s, plus a
  pilot stream at 11.4 m/s;
* local time step dt = CFL min(dx / u, dx^2 / (4 D)) per cell;
* the initial field carries the inflow profile along x (each row its
  stream), so pilot and jet start to mix and ignite at their interface.
"""
from __future__ import annotations

import numpy as np

from .cells import equilibrium_tp, mole_to_mass
from .mechgen import standard_mechanism

P_ATM = 101325.0


def _mass_fractions(mech, moles):
    W = mech.molar_masses()
    x = np.zeros(mech.n_species)
    for name, v in moles.items():
        x[mech.index(name)] = v
    y = x * W
    return y / y.sum()


def flame_field(nx=170, ny=170, dx=1.0e-3, D=2.0e-4, cfl=0.5, seed=301):
    mech = standard_mechanism("chon_53")
    N = mech.n_species
    rng = np.random.default_rng(seed)
    y_c = (np.arange(ny) - (ny - 1) / 2.0) * dx
    x_c = (np.arange(nx) + 0.5) * dx
    # streams (volume fractions as mole fractions)
    jet = _mass_fractions(mech, {"CH4": 0.20, "NH3": 0.05, "O2": 0.157, "N2": 0.593})
    air = _mass_fractions(mech, {"O2": 0.21, "N2": 0.79})
    lean = _mass_fractions(mech, {"CH4": 0.04, "NH3": 0.01, "O2": 0.20, "N2": 0.75})
    A = mech.element_matrix()
    b = (lean / mech.molar_masses()) @ A.T
    pilot = mole_to_mass(mech, equilibrium_tp(mech, np.array([1880.0]), np.array([P_ATM]), b[None, :]))[0]
    ay = np.abs(y_c)
    stream = np.where(ay < 3.6e-3, 0, np.where(ay < 9.1e-3, 1, 2))
    Yin = np.stack([jet, pilot, air])[stream]          # [ny, N]
    Tin = np.array([294.0, 1880.0, 291.0])[stream]
    # small seeded perturbation of the jet composition (keeps cells distinct)
    Yin = Yin * (1.0 + 1e-3 * rng.standard_normal(Yin.shape) * (Yin > 0))
    Yin /= Yin.sum(1, keepdims=True)
    # velocity
    b0, Uj, Uc, Up = 3.6e-3, 49.6, 0.9, 11.4
    bx = b0 + 0.08 * x_c[None, :]
    u = Uc + (Uj - Uc) * (b0 / bx) * np.exp(-(y_c[:, None] / bx) ** 2)
    u += (Up - Uc) * np.exp(-((ay[:, None] - 6.5e-3) / 2.5e-3) ** 2) * (b0 / bx)
    dt = cfl * np.minimum(dx / u, dx * dx / (4.0 * D))
    # state, cells row-major (c = iy*nx + ix)
    T = np.repeat(Tin, nx)
    Y = np.repeat(Yin, nx, axis=0)                     # [ny*nx, N]
    return dict(mech=mech, nx=nx, ny=ny, dx=dx, D=D, T=T, p=np.full(nx * ny, P_ATM), Y=Y,
                u=u.reshape(-1), dt=dt.reshape(-1), inflow_T=Tin, inflow_Y=Yin.T.copy(),
                stream=np.repeat(stream, nx), N=N, Y_fuel=jet, Y_ox=air)


def mixing_cells(n=512, seed=302):
    """Cells of the flame's mixing layers, for the reference-cell mapping:
    the jet and air streams of flame_field (the mapping's fuel and
    oxidiser), and per cell one of
      * coflow air at 291 K plus 0-2 K (40%),
      * air with a trace of jet or pilot gas, mass fraction 10^U[-6,-2.7],
        at 291-300 K (25%),
      * a jet/air mixture of jet fraction U[0,1] at the mixing temperature of
        the two streams (20%),
      * pilot gas (the 1880 K burnt lean mixture of flame_field) mixed with
        up to 30% air, at 1500-1880 K (15%);
    1 atm, local dt log-uniform over the flame field's range (1e-5 to
    5.6e-4 s).  Rows of Y are [n, N]."""
    f = flame_field(nx=2, ny=170)
    mech = f["mech"]
    jet, air = f["Y_fuel"], f["Y_ox"]
    pilot = f["inflow_Y"][:, f["inflow_T"] > 1000.0][:, 0]
    rng = np.random.default_rng(seed)
    kind = rng.choice(4, size=n, p=[0.40, 0.25, 0.20, 0.15])
    Y = np.empty((n, mech.n_species))
    T = np.empty(n)
    for c in range(n):
        if kind[c] == 0:
            Y[c], T[c] = air, 291.0 + 2.0 * rng.uniform()
        elif kind[c] == 1:
            a = 10.0 ** rng.uniform(-6.0, -2.7)
            src = jet if rng.uniform() < 0.5 else pilot
            Y[c], T[c] = a * src + (1 - a) * air, 291.0 + 9.0 * rng.uniform()
        elif kind[c] == 2:
            a = rng.uniform()
            Y[c], T[c] = a * jet + (1 - a) * air, 294.0 * a + 291.0 * (1 - a)
        else:
            a = rng.uniform(0.0, 0.3)
            Y[c], T[c] = a * air + (1 - a) * pilot, rng.uniform(1500.0, 1880.0)
    dt = 10.0 ** rng.uniform(-5.0, np.log10(5.6e-4), n)
    return dict(mech=mech, T=T, p=np.full(n, P_ATM), Y=Y, dt=dt, kind=kind, Y_fuel=jet, Y_ox=air)
