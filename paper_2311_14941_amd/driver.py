"""Operator-split driver with local time stepping (paper Sec. 2.5), with
optional zonal reference-cell mapping of the chemistry.

Each split step integrates the chemistry of every cell of a 2-D grid over
that cell's own time step (a CFL-limited local step, so the batch is
uneven), then applies one explicit transport update (upwind advection along
x plus diffusion, sc_transport2d) to the mass fractions and the
temperature.  The persistent queue with the previous step's per-cell step
counts as the cost order is the natural launch here: the counts of one
split step predict the next.  The step size h of every cell carries from
one split step to the next.

State layout: one [N + 1, cells] float64 array, rows 0..N-1 the mass
fractions and row N the temperature, so chemistry reads Y and T as views
and transport updates all N + 1 rows in one launch.  Two such arrays
alternate; nothing is allocated per step.
"""
from __future__ import annotations

from . import Plan, _check, _ptr, _stream, lib


class SplitDriver:
    """Chemistry + transport split steps on an nx x ny grid (cells
    row-major, c = iy*nx + ix).

    plan          a Plan of the mechanism (its launch configuration is used)
    p, u, dt      per-cell pressure [Pa], x-velocity [m/s] (>= 0) and local
                  time step [s]; dt must satisfy u dt/dx + 4 D dt/dx^2 <= 1
                  for the transport update to stay bounded
    dx, diffusivity  grid spacing [m] and diffusion coefficient [m^2/s]
    inflow_T, inflow_Y  inflow profile at x = 0: [ny] and [N, ny]
    mapping       None, or a dict (Y_fuel, Y_ox, z_tol, dT, dlnp) for zonal
                  reference-cell mapping of the chemistry (Plan.set_mapping):
                  low-reactivity cells take their zone reference's change
    """

    def __init__(self, plan: Plan, nx, ny, p, u, dt, dx, diffusivity, inflow_T, inflow_Y, mapping=None):
        t = plan.torch
        self.plan, self.nx, self.ny = plan, int(nx), int(ny)
        n = self.nx * self.ny
        N = plan.mech.N
        self.n, self.N = n, N
        self.p = plan._dev(p)
        if self.p.dim() == 0:
            self.p = self.p.expand(n).contiguous()
        self.u, self.dt = plan._dev(u), plan._dev(dt)
        if self.u.shape != (n,) or self.dt.shape != (n,) or self.p.shape != (n,):
            raise ValueError("p, u and dt need one value per cell")
        self.dx, self.D = float(dx), float(diffusivity)
        co = (self.u * self.dt / self.dx + 4.0 * self.D * self.dt / self.dx ** 2)
        if bool((self.u < 0).any()) or bool((co > 1.0 + 1e-12).any()):
            raise ValueError("need u >= 0 and u dt/dx + 4 D dt/dx^2 <= 1 in every cell")
        infY = plan._dev(inflow_Y)
        infT = plan._dev(inflow_T)
        if infY.shape != (N, self.ny) or infT.shape != (self.ny,):
            raise ValueError("inflow_Y must be [N, ny] and inflow_T [ny]")
        self.inflow = t.cat([infY, infT[None, :]]).contiguous()
        dev = self.p.device
        self.q = [t.empty(N + 1, n, dtype=t.float64, device=dev) for _ in range(2)]
        self.h = t.zeros(n, dtype=t.float64, device=dev)
        mk = lambda: t.zeros(n, dtype=t.int32, device=dev)
        self.status, self.n_acc, self.n_rej = mk(), mk(), mk()
        self.steps = t.zeros(n, dtype=t.int64, device=dev)
        self.failed = t.zeros(n, dtype=t.int64, device=dev)
        self.ref = None
        if mapping is not None:
            plan.set_mapping(mapping["Y_fuel"], mapping["Y_ox"], mapping["z_tol"], mapping["dT"],
                             mapping.get("dlnp", 0.0))
            self.ref = t.empty(n, dtype=t.int32, device=dev)

    def load(self, T, Y, h=None):
        """Set the state: T [cells], Y [N, cells]; step sizes restart unless h is given."""
        self.q[0][self.N].copy_(self.plan._dev(T))
        self.q[0][:self.N].copy_(self.plan._dev(Y))
        self.h.zero_() if h is None else self.h.copy_(self.plan._dev(h))
        self.steps.zero_()
        self.failed.zero_()

    def chemistry(self):
        """Integrate every cell over its dt: q[0] -> q[1]."""
        a, b, N, n = self.q[0], self.q[1], self.N, self.n
        plan = self.plan
        args = (plan._h, n, _ptr(a[N]), _ptr(self.p), _ptr(a[:N]), n, _ptr(self.dt), None, _ptr(self.h),
                _ptr(b[N]), _ptr(b[:N]), _ptr(self.status), _ptr(self.n_acc), _ptr(self.n_rej))
        if self.ref is None:
            _check(lib().sc_integrate(*args, _stream(plan.torch, plan.device)))
        else:
            _check(lib().sc_integrate_mapped(*args, _ptr(self.ref), _stream(plan.torch, plan.device)))
        self.steps.add_(self.n_acc).add_(self.n_rej)
        self.failed.add_((self.status != 0).long())

    def transport(self):
        """One transport update of all N + 1 rows: q[1] -> q[0]."""
        plan = self.plan
        _check(lib().sc_transport2d(self.nx, self.ny, self.N + 1, _ptr(self.q[1]), self.n, _ptr(self.u),
                                    _ptr(self.dt), self.dx, self.D, _ptr(self.inflow), _ptr(self.q[0]),
                                    _stream(plan.torch, plan.device)))

    def step(self, k=1):
        for _ in range(k):
            self.chemistry()
            self.transport()

    @property
    def T(self):
        return self.q[0][self.N]

    @property
    def Y(self):
        return self.q[0][:self.N]
