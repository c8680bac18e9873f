"""Argument checks of the Python binding: every per-cell array reaching a
kernel must have one entry per cell (the kernels index them up to n), so a
wrong shape is a ValueError before any launch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    import paper_2311_14941_amd as sc
    from synth.cells import make_cells
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    sc.ensure_built()
    c = make_cells("C1", n=16)
    d = "cuda:0"
    T = torch.tensor(c["T"], device=d)
    p = torch.tensor(c["p"], device=d)
    Y = torch.tensor(np.ascontiguousarray(c["Y"].T), device=d)
    dt = torch.tensor(c["dt"], device=d)
    plan = sc.Plan(sc.Mechanism(c["mech"].to_text()))
    return torch, sc, plan, T, p, Y, dt


def test_short_per_cell_arrays_are_rejected(setup):
    torch, sc, plan, T, p, Y, dt = setup
    with pytest.raises(ValueError, match="dt"):
        plan.integrate(T, p, Y, dt[:8])
    with pytest.raises(ValueError, match="p"):
        plan.integrate(T, p[:8], Y, dt)
    with pytest.raises(ValueError, match="h"):
        plan.integrate(T, p, Y, dt, h=torch.zeros(3, dtype=torch.float64, device="cuda:0"))
    with pytest.raises(ValueError, match="Y"):
        plan.integrate(T, p, Y[:, :8], dt)
    with pytest.raises(ValueError, match="b"):
        plan.linsolve(T, p, Y, 1e-6, torch.zeros(16, 3, dtype=torch.float64, device="cuda:0"))
    with pytest.raises(ValueError, match="dt"):
        plan.adjoint(T, p, Y, dt[:4], torch.ones_like(T), torch.zeros_like(Y))
    with pytest.raises(ValueError, match="cost"):
        plan.adjoint(T, p, Y, dt, torch.ones_like(T), torch.zeros_like(Y),
                     cost=torch.zeros(5, dtype=torch.int32, device="cuda:0"))


def test_scalar_arguments_broadcast_and_out_is_checked(setup):
    torch, sc, plan, T, p, Y, dt = setup
    a = plan.integrate(T, 101325.0, Y, 1e-5)
    b = plan.integrate(T, torch.full_like(T, 101325.0), Y, torch.full_like(T, 1e-5))
    assert torch.equal(a["T"], b["T"]) and torch.equal(a["Y"], b["Y"])
    bad = dict(a)
    bad["n_acc"] = torch.zeros(3, dtype=torch.int32, device="cuda:0")
    with pytest.raises(ValueError, match="n_acc"):
        plan.integrate(T, p, Y, dt, out=bad)


def test_transport_shapes_are_checked(setup):
    torch, sc, plan, T, p, Y, dt = setup
    q = torch.zeros(2, 12, dtype=torch.float64, device="cuda:0")
    u = torch.zeros(12, dtype=torch.float64, device="cuda:0")
    inflow = torch.zeros(2, 3, dtype=torch.float64, device="cuda:0")
    sc.transport2d(4, 3, q, u, u, 1e-3, 0.0, inflow)
    with pytest.raises(ValueError):
        sc.transport2d(4, 3, q, u[:6], u, 1e-3, 0.0, inflow)
    with pytest.raises(ValueError):
        sc.transport2d(4, 3, q, u, u, 1e-3, 0.0, inflow, out=torch.zeros(2, 6, dtype=torch.float64,
                                                                          device="cuda:0"))
